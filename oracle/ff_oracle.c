/*
 * ff_oracle.c -- plain, slow CPU oracle of the Flow Fields hot path
 * (Bailer, Taetz, Stricker, "Flow Fields: Dense Correspondence Fields for
 * Highly Accurate Large Displacement Optical Flow Estimation").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; it is written from the paper's
 * description of the method, in the paper's order, with plain scalar loops.
 *
 * What it computes (readings of the paper are marked R#, listed in full in
 * the design notes of the repository):
 *   blur        scale-space low-pass I^n (Sec. 3.2; Sec. 3.6 low-pass and
 *               replicate border), R12: integer box filter of half-width
 *               max(1, n/2), rounded half up.
 *   descriptor  per-pixel 16-byte feature of I^n: 4x4 samples with spacing 2n
 *               (F2 reading of Sec. 3.6, features taken after low-pass), R13.
 *   cost        matching error E_n of the subsampled patch P^n_r (Eq. 3):
 *               sum over (2r+1)^2 patch positions of the byte-wise SAD of the
 *               two descriptors, replicate border at every read.
 *   nn          exact nearest neighbour of every coarsest-grid pixel over all
 *               pixels of the other image under squared L2 of the level-1
 *               descriptors (stands in for the kd-tree of Sec. 3.1 with leaf
 *               size 1, R4); ties go to the smallest linear index.
 *   nn_topl     the l nearest pixels in the same order (the candidate set L
 *               of Sec. 3.1 read as the l nearest neighbours, R28); with a
 *               reference step of 2, the even pixels only (Fast x2, R30).
 *   init        initial flow F = q - p (Eq. 1 / Eq. 4) and its cost at the
 *               coarsest scale: the candidate of lowest E_nc, the earlier
 *               rank on equal cost (|L| = 1: the nearest neighbour).
 *   seed_level  coarse-to-fine hand-over (Sec. 3.2): grid pixels shared with
 *               the coarser grid keep its flow (same full-resolution pixel)
 *               and re-evaluate the cost; all others start UNSET.
 *   propagate   one propagation step (Eq. 2) in direction d = pass mod 4
 *               (R2: d cycle right-down, left-up, left-down, right-up) run
 *               as two checkerboard half-sweeps (R1), odd (i+j) first (R11);
 *               candidate order own, horizontal, vertical, strict "<" (R3);
 *               candidates whose target leaves the image are rejected (R9).
 *   propagate_raster  the same step in the serial order of Sec. 3.1 (a cell
 *               after its two source cells), R29.
 *   random_search  one random-search step (Sec. 3.1) with integer offsets
 *               uniform on [-R_n, R_n]^2, R_n = floor(R * n) (R5, R6), drawn
 *               from a counter-based generator: SplitMix64's output mixer
 *               (Steele, Lea, Flood, OOPSLA 2014) applied as
 *               mix(seed ^ mix(counter)), mapped to a range by Lemire's
 *               multiply-shift (ACM TOMACS 2019).
 *   consistency forward-backward check (Sec. 3.7): keep p iff
 *               |F(p) + F_b(p + F(p))| < eps, evaluated exactly (R14);
 *               consistency2 the same against two backward fields;
 *               consistency_grid the check of fields on the grid of scale
 *               n (one match per n x n region, Fast x2, R30).
 *   region_filter  deletes small regions next to removed outliers (Sec. 3.7).
 *   sparsify    one sample per q x q region (Sec. 3.8).
 *   cost_sub    the subpixel form (Sec. 3.1: random-search offsets with
 *               subpixel accuracy, colours by bilinear interpolation): flows
 *               in units of 1/2^s pixel, image b's descriptors bilinearly
 *               interpolated at the target, costs scaled by 4^s (exact).
 *   flow_fields the whole multi-scale schedule (Sec. 3.1, 3.2): L levels
 *               n = 2^(L-1) .. 1, T propagation steps per level with T-1
 *               random-search steps between them, forward and backward;
 *               optionally the Flow Fields+ steps (Sec. 3.3: P steps at
 *               R^+ first), the Fast finest scale (Sec. 3.4), Fast x2
 *               (finest scale skipped, R30) and sub-scales (Sec. 3.3, R31:
 *               patch scales 3n/2 on the grid of scale n; rescore moves a
 *               grid to another patch scale).
 *
 * Layouts: images uint8 [H][W]; descriptors uint8 [H][W][16]; a level grid
 * of scale n has ceil(W/n) x ceil(H/n) cells, cell (i, j) <-> pixel
 * (i*n, j*n); flows int16 [cells][2] (dx, dy); costs uint32 [cells] with
 * 0xFFFFFFFF = UNSET (its flow is (0, 0)).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_UNSET 0xFFFFFFFFu

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int ceil_div(int a, int b) { return (a + b - 1) / b; }

int or_version(void) { return 1; }

/* Scale-space image I^n (Sec. 3.2 scale spaces; Sec. 3.6 low-pass; Sec. 3.6
 * border condition): every output pixel is the rounded mean of the
 * (2h+1)x(2h+1) window around it, h = max(1, n/2), pixels outside the image
 * replaced by the nearest inside pixel. */
void or_blur(const uint8_t *img, int W, int H, int n, uint8_t *out)
{
    int h = n / 2 < 1 ? 1 : n / 2;
    int64_t area = (int64_t)(2 * h + 1) * (2 * h + 1);
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t s = 0;
            for (int dy = -h; dy <= h; ++dy)
                for (int dx = -h; dx <= h; ++dx)
                    s += img[(size_t)clampi(y + dy, 0, H - 1) * W + clampi(x + dx, 0, W - 1)];
            out[(size_t)y * W + x] = (uint8_t)((s + area / 2) / area);
        }
}

/* Per-pixel feature of scale n: 16 samples of I^n on a 4x4 grid with spacing
 * 2n centred on the pixel, channel 4*gy + gx <-> offset n*(2gx-3, 2gy-3),
 * replicate border. */
void or_descriptor(const uint8_t *blurred, int W, int H, int n, uint8_t *desc)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int gy = 0; gy < 4; ++gy)
                for (int gx = 0; gx < 4; ++gx) {
                    int sx = clampi(x + n * (2 * gx - 3), 0, W - 1);
                    int sy = clampi(y + n * (2 * gy - 3), 0, H - 1);
                    desc[((size_t)y * W + x) * 16 + 4 * gy + gx] = blurred[(size_t)sy * W + sx];
                }
}

/* Matching error E_n(p, f) of the subsampled patch P^n_r (Eq. 3): every n-th
 * pixel within radius r*n of p in image a against the same pattern around
 * p + f in image b; each patch position contributes the sum of absolute
 * differences of the two 16-byte descriptors; reads outside the image take
 * the nearest inside pixel. */
uint32_t or_cost(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int r,
                 int x, int y, int fx, int fy)
{
    uint32_t s = 0;
    for (int v = -r; v <= r; ++v)
        for (int u = -r; u <= r; ++u) {
            int ax = clampi(x + n * u, 0, W - 1), ay = clampi(y + n * v, 0, H - 1);
            int bx = clampi(x + fx + n * u, 0, W - 1), by = clampi(y + fy + n * v, 0, H - 1);
            const uint8_t *a = Da + ((size_t)ay * W + ax) * 16;
            const uint8_t *b = Db + ((size_t)by * W + bx) * 16;
            for (int c = 0; c < 16; ++c)
                s += (uint32_t)abs((int)a[c] - (int)b[c]);
        }
    return s;
}

/* A matching error as an unsigned 32-bit key: the integer SAD itself, or
 * the bit pattern of a non-negative float cost (non-negative IEEE-754
 * singles order exactly like their bit patterns), so one schedule serves
 * both data terms.  0xFFFFFFFF (UNSET) is above every such value. */
typedef uint32_t (*or_cost_fn)(const void *A, const void *B, int W, int H, int n, int r, int x, int y, int fx,
                               int fy, int s);

static uint32_t cost_u8(const void *A, const void *B, int W, int H, int n, int r, int x, int y, int fx, int fy,
                        int s)
{
    (void)s;
    return or_cost((const uint8_t *)A, (const uint8_t *)B, W, H, n, r, x, y, fx, fy);
}

/* Learned-feature matching error (Sec. 3.5 learned data term, read as the
 * sum of squared differences of 16-channel float features over the
 * subsampled patch of Eq. 3, replicate border), in single precision, R18:
 * one partial sum per group of four channels (g = 0..3: channels 4g..4g+3),
 * each accumulated by one fused multiply-add per term in the order v, u, c;
 * the four partial sums are then added as (s0 + s1) + (s2 + s3). */
uint32_t or_cost_f32(const float *fa, const float *fb, int W, int H, int n, int r, int x, int y, int fx, int fy)
{
    float part[4];
    for (int g = 0; g < 4; ++g) {
        float acc = 0.0f;
        for (int v = -r; v <= r; ++v)
            for (int u = -r; u <= r; ++u) {
                int ax = clampi(x + n * u, 0, W - 1), ay = clampi(y + n * v, 0, H - 1);
                int bx = clampi(x + fx + n * u, 0, W - 1), by = clampi(y + fy + n * v, 0, H - 1);
                const float *a = fa + ((size_t)ay * W + ax) * 16;
                const float *b = fb + ((size_t)by * W + bx) * 16;
                for (int c = 4 * g; c < 4 * g + 4; ++c) {
                    float d = a[c] - b[c];
                    acc = fmaf(d, d, acc);
                }
            }
        part[g] = acc;
    }
    float total = (part[0] + part[1]) + (part[2] + part[3]);
    uint32_t bits;
    memcpy(&bits, &total, sizeof bits);
    return bits;
}

static uint32_t cost_f32(const void *A, const void *B, int W, int H, int n, int r, int x, int y, int fx, int fy,
                         int s)
{
    (void)s;
    return or_cost_f32((const float *)A, (const float *)B, W, H, n, r, x, y, fx, fy);
}

/* Matching error of a subpixel flow (Sec. 3.1: random-search offsets with
 * subpixel accuracy; the colours of the target patch by bilinear
 * interpolation).  Flows are in units of 1/2^s pixel, S = 2^s: the target
 * t = p + f / S lies in the cell of the integer pixels (tx0, ty0) ..
 * (tx0 + 1, ty0 + 1) with fractions ax, ay in [0, S); the descriptors of
 * image b at every patch position t + n(u, v) are the bilinear mix of those
 * four pixels' descriptors (each read through the border, as or_cost does)
 * with weights (S - ax)(S - ay), ax (S - ay), (S - ax) ay, ax ay, which sum
 * to S^2.  The error is sum |S^2 a - sum_k w_k b_k| over the patch positions
 * and channels: the cost of Eq. 3 on the interpolated descriptors times
 * S^2, an exact integer (for an integer flow, S^2 times or_cost).  The
 * target must lie in the image (0 <= t <= W - 1, 0 <= t_y <= H - 1). */
uint32_t or_cost_sub(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int r, int x, int y, int fx, int fy,
                     int s)
{
    int S = 1 << s;
    int tx = x * S + fx, ty = y * S + fy;
    int tx0 = tx / S, ty0 = ty / S, ax = tx - tx0 * S, ay = ty - ty0 * S;
    int w[4] = {(S - ax) * (S - ay), ax * (S - ay), (S - ax) * ay, ax * ay};
    int cx[4] = {tx0, tx0 + 1, tx0, tx0 + 1}, cy[4] = {ty0, ty0, ty0 + 1, ty0 + 1};
    uint32_t sum = 0;
    for (int v = -r; v <= r; ++v)
        for (int u = -r; u <= r; ++u) {
            int ax_ = clampi(x + n * u, 0, W - 1), ay_ = clampi(y + n * v, 0, H - 1);
            const uint8_t *a = Da + ((size_t)ay_ * W + ax_) * 16;
            const uint8_t *b[4];
            for (int k = 0; k < 4; ++k) {
                int bx = clampi(cx[k] + n * u, 0, W - 1), by = clampi(cy[k] + n * v, 0, H - 1);
                b[k] = Db + ((size_t)by * W + bx) * 16;
            }
            for (int c = 0; c < 16; ++c) {
                int mix = 0;
                for (int k = 0; k < 4; ++k) mix += w[k] * b[k][c];
                sum += (uint32_t)abs(S * S * (int)a[c] - mix);
            }
        }
    return sum;
}

static uint32_t cost_u8_sub(const void *A, const void *B, int W, int H, int n, int r, int x, int y, int fx, int fy,
                            int s)
{
    return or_cost_sub((const uint8_t *)A, (const uint8_t *)B, W, H, n, r, x, y, fx, fy, s);
}

/* Target p + f / 2^s of a flow lies in the image. */
static int target_in(int W, int H, int x, int y, int fx, int fy, int s)
{
    int tx = x * (1 << s) + fx, ty = y * (1 << s) + fy;
    return tx >= 0 && tx <= (W - 1) * (1 << s) && ty >= 0 && ty <= (H - 1) * (1 << s);
}

/* Learned features to bytes for the NN seed: with lo, hi the range of all
 * values, q = clamp(rint((f - lo) * (255 / (hi - lo))), 0, 255) in single
 * precision. */
static void quantize_range(const float *f, int64_t count, float lo, float hi, uint8_t *q)
{
    float s = hi > lo ? 255.0f / (hi - lo) : 0.0f;
    for (int64_t i = 0; i < count; ++i) {
        float t = rintf((f[i] - lo) * s);
        q[i] = (uint8_t)fminf(fmaxf(t, 0.0f), 255.0f);
    }
}

static void value_range(const float *f, int64_t count, float *lo, float *hi)
{
    for (int64_t i = 0; i < count; ++i) {
        *lo = fminf(*lo, f[i]);
        *hi = fmaxf(*hi, f[i]);
    }
}

void or_quantize_u8(const float *f, int64_t count, uint8_t *q)
{
    float lo = INFINITY, hi = -INFINITY;
    value_range(f, count, &lo, &hi);
    quantize_range(f, count, lo, hi, q);
}

/* Both images' level-1 features with ONE range (lo, hi over both maps), so
 * that equal feature values become equal bytes in both images and the
 * byte-space nearest neighbour is taken on one scale (Sec. 3.1: the seed is
 * the nearest neighbour in feature space). */
void or_quantize_pair_u8(const float *f1, const float *f2, int64_t count, uint8_t *q1, uint8_t *q2)
{
    float lo = INFINITY, hi = -INFINITY;
    value_range(f1, count, &lo, &hi);
    value_range(f2, count, &lo, &hi);
    quantize_range(f1, count, lo, hi, q1);
    quantize_range(f2, count, lo, hi, q2);
}

/* Exact nearest neighbour (stands in for the kd-tree candidate set of
 * Sec. 3.1): for every cell of the grid of scale nc, the pixel q of image b
 * whose level-1 descriptor has the smallest squared L2 distance to the
 * cell's pixel descriptor in image a; ties -> smallest q.y*W + q.x. */
void or_nn(const uint8_t *Da1, const uint8_t *Db1, int W, int H, int nc,
           int32_t *best_idx, int64_t *best_dist, int nthreads)
{
    int Wc = ceil_div(W, nc), Hc = ceil_div(H, nc);
    int64_t N = (int64_t)W * H;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int k = 0; k < Wc * Hc; ++k) {
        int i = k % Wc, j = k / Wc;
        const uint8_t *a = Da1 + ((size_t)(j * nc) * W + (size_t)(i * nc)) * 16;
        int64_t bd = INT64_MAX;
        int32_t bi = -1;
        for (int64_t q = 0; q < N; ++q) {
            const uint8_t *b = Db1 + (size_t)q * 16;
            int64_t d = 0;
            for (int c = 0; c < 16; ++c) {
                int64_t e = (int64_t)a[c] - (int64_t)b[c];
                d += e * e;
            }
            if (d < bd) { bd = d; bi = (int32_t)q; }
        }
        best_idx[k] = bi;
        best_dist[k] = bd;
    }
}

/* The l nearest neighbours (the candidate set L of Sec. 3.1, a kd-tree leaf
 * of size l, read as the l nearest pixels): for every cell of the grid of
 * scale nc, the l pixels q of image b with the smallest (squared L2 distance
 * of the level-1 descriptors, q.y*W + q.x), in that order; idx[k*l + c],
 * dist[k*l + c] is candidate c of cell k, idx -1 (dist INT64_MAX) where the
 * image has fewer than l pixels.  l = 1 is or_nn.  rstep = 2: only the
 * pixels with even x and y are candidates (Flow Fields+ Fast x2, Sec. 3.4:
 * one pixel of every 2x2 region enters the tree). */
void or_nn_topl_step(const uint8_t *Da1, const uint8_t *Db1, int W, int H, int nc, int l, int rstep,
                     int32_t *idx, int64_t *dist, int nthreads)
{
    int Wc = ceil_div(W, nc), Hc = ceil_div(H, nc);
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int k = 0; k < Wc * Hc; ++k) {
        int i = k % Wc, j = k / Wc;
        const uint8_t *a = Da1 + ((size_t)(j * nc) * W + (size_t)(i * nc)) * 16;
        int32_t *bi = idx + (size_t)k * l;
        int64_t *bd = dist + (size_t)k * l;
        for (int c = 0; c < l; ++c) { bi[c] = -1; bd[c] = INT64_MAX; }
        for (int qy = 0; qy < H; qy += rstep)
            for (int qx = 0; qx < W; qx += rstep) {
                int32_t q = qy * W + qx;
                const uint8_t *b = Db1 + (size_t)q * 16;
                int64_t d = 0;
                for (int c = 0; c < 16; ++c) {
                    int64_t e = (int64_t)a[c] - (int64_t)b[c];
                    d += e * e;
                }
                /* q grows, so an equal distance ranks after every listed entry */
                if (d >= bd[l - 1]) continue;
                int pos = l - 1;
                while (pos > 0 && bd[pos - 1] > d) {
                    bd[pos] = bd[pos - 1];
                    bi[pos] = bi[pos - 1];
                    --pos;
                }
                bd[pos] = d;
                bi[pos] = q;
            }
    }
}

void or_nn_topl(const uint8_t *Da1, const uint8_t *Db1, int W, int H, int nc, int l,
                int32_t *idx, int64_t *dist, int nthreads)
{
    or_nn_topl_step(Da1, Db1, W, H, nc, l, 1, idx, dist, nthreads);
}

/* Initial flow of the coarsest scale (Eq. 1; Eq. 4 at scale nc): of the l
 * candidates q of a cell p (idx[k*l + c], in rank order, -1 = none), the one
 * with the lowest E_nc(p, q - p), the earlier rank on equal cost; every
 * candidate costs one evaluation.  F(p) = q - p. */
static void init_coarse_g(or_cost_fn E, int s, const int32_t *best_idx, int l, const void *Da, const void *Db, int W,
                          int H, int nc, int m, int r, int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    int Wc = ceil_div(W, nc), Hc = ceil_div(H, nc);
    for (int j = 0; j < Hc; ++j)
        for (int i = 0; i < Wc; ++i) {
            int k = j * Wc + i, x = i * nc, y = j * nc;
            uint32_t bc = OR_UNSET;
            int bfx = 0, bfy = 0, have = 0;
            for (int c = 0; c < l; ++c) {
                int32_t q = best_idx[(size_t)k * l + c];
                if (q < 0) continue;
                int fx = (q % W - x) * (1 << s), fy = (q / W - y) * (1 << s);  /* integer seed, in 1/2^s pixel */
                uint32_t e = E(Da, Db, W, H, m, r, x, y, fx, fy, s);
                *n_evals += 1;
                if (!have || e < bc) { bc = e; bfx = fx; bfy = fy; have = 1; }
            }
            flow[2 * k] = (int16_t)bfx;
            flow[2 * k + 1] = (int16_t)bfy;
            cost[k] = bc;
        }
}

void or_init_coarse(const int32_t *best_idx, const uint8_t *Da, const uint8_t *Db, int W, int H,
                    int nc, int r, int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    init_coarse_g(cost_u8, 0, best_idx, 1, Da, Db, W, H, nc, nc, r, flow, cost, n_evals);
}

void or_init_coarse_l(const int32_t *cand_idx, int l, const uint8_t *Da, const uint8_t *Db, int W, int H,
                      int nc, int r, int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    init_coarse_g(cost_u8, 0, cand_idx, l, Da, Db, W, H, nc, nc, r, flow, cost, n_evals);
}

/* Hand-over from scale 2n to scale n (Sec. 3.2): cell (i, j) with i and j
 * even is the same full-resolution pixel as coarse cell (i/2, j/2) and takes
 * its flow as a seed (flows are kept in full-resolution pixel units); its
 * cost is re-evaluated with E_n.  All other cells start UNSET and receive a
 * value in the first propagation step. */
static void seed_level_g(or_cost_fn E, int s, const int16_t *cflow, const uint32_t *ccost, const void *Da,
                         const void *Db, int W, int H, int n, int m, int r, int16_t *flow, uint32_t *cost,
                         uint64_t *n_evals)
{
    int Wn = ceil_div(W, n), Hn = ceil_div(H, n), Wc = ceil_div(W, 2 * n);
    for (int j = 0; j < Hn; ++j)
        for (int i = 0; i < Wn; ++i) {
            int k = j * Wn + i;
            flow[2 * k] = 0;
            flow[2 * k + 1] = 0;
            cost[k] = OR_UNSET;
            if ((i & 1) || (j & 1)) continue;
            int kc = (j / 2) * Wc + i / 2;
            if (ccost[kc] == OR_UNSET) continue;
            int fx = cflow[2 * kc], fy = cflow[2 * kc + 1];
            flow[2 * k] = (int16_t)fx;
            flow[2 * k + 1] = (int16_t)fy;
            cost[k] = E(Da, Db, W, H, m, r, i * n, j * n, fx, fy, s);
            *n_evals += 1;
        }
}

void or_seed_level(const int16_t *cflow, const uint32_t *ccost, const uint8_t *Da, const uint8_t *Db,
                   int W, int H, int n, int r, int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    seed_level_g(cost_u8, 0, cflow, ccost, Da, Db, W, H, n, n, r, flow, cost, n_evals);
}

/* Source cells of propagation direction d (Eq. 2 for d = 0; the other three
 * quadrants for d = 1..3). */
static void prop_sources(int d, int *hdi, int *vdj)
{
    static const int H_[4] = {-1, +1, +1, -1};
    static const int V_[4] = {-1, +1, -1, +1};
    *hdi = H_[d & 3];
    *vdj = V_[d & 3];
}

/* One propagation step (Eq. 2) at scale n: for every cell the flow is the
 * best of its own flow and the flows of its horizontal and vertical source
 * cells, by E_n with strict improvement.  Run as two half-sweeps: first all
 * cells with (i+j) odd, then all with (i+j) even; a cell only reads cells of
 * the other colour, so the result does not depend on the visiting order. */
static void propagate_g(or_cost_fn E, int s, const void *Da, const void *Db, int W, int H, int n, int m, int r,
                        int pass, int16_t *flow, uint32_t *cost, uint64_t *n_evals, int nthreads)
{
    int Wn = ceil_div(W, n), Hn = ceil_div(H, n), hdi, vdj;
    prop_sources(pass & 3, &hdi, &vdj);
    (void)nthreads;
    for (int colour = 1; colour >= 0; --colour) {
        uint64_t cnt = 0;
#ifdef _OPENMP
#pragma omp parallel for reduction(+ : cnt) schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
        for (int j = 0; j < Hn; ++j)
            for (int i = 0; i < Wn; ++i) {
                if (((i + j) & 1) != colour) continue;
                int k = j * Wn + i, x = i * n, y = j * n;
                uint32_t bc = cost[k];
                int bfx = flow[2 * k], bfy = flow[2 * k + 1];
                for (int src = 0; src < 2; ++src) {  /* horizontal, then vertical source */
                    int si = src == 0 ? i + hdi : i, sj = src == 0 ? j : j + vdj;
                    if (si < 0 || si >= Wn || sj < 0 || sj >= Hn) continue;
                    int ks = sj * Wn + si;
                    if (cost[ks] == OR_UNSET) continue;
                    int fx = flow[2 * ks], fy = flow[2 * ks + 1];
                    if (bc != OR_UNSET && fx == bfx && fy == bfy) continue;
                    if (!target_in(W, H, x, y, fx, fy, s)) continue;
                    uint32_t e = E(Da, Db, W, H, m, r, x, y, fx, fy, s);
                    cnt += 1;
                    if (e < bc) { bc = e; bfx = fx; bfy = fy; }
                }
                cost[k] = bc;
                flow[2 * k] = (int16_t)bfx;
                flow[2 * k + 1] = (int16_t)bfy;
            }
        *n_evals += cnt;
    }
}

void or_propagate(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int r, int pass,
                  int16_t *flow, uint32_t *cost, uint64_t *n_evals, int nthreads)
{
    propagate_g(cost_u8, 0, Da, Db, W, H, n, n, r, pass, flow, cost, n_evals, nthreads);
}

/* One propagation step (Eq. 2) in the serial order the paper asks for: a
 * cell is updated only after its horizontal and vertical source cells, so a
 * flow can travel any distance within the step's quadrant.  Direction d's
 * sources sit at (i + hdi, j) and (i, j + vdj); the scan takes the rows
 * starting from the side of the vertical source and, within a row, the
 * cells starting from the side of the horizontal source (d = 0: ordinary
 * raster order).  The per-cell update is that
 * of the checkerboard step (own, horizontal, vertical; strictly lower wins;
 * UNSET, held and out-of-image candidates skipped), reading the sources'
 * values of this step. */
static void propagate_raster_g(or_cost_fn E, int s, const void *Da, const void *Db, int W, int H, int n, int m,
                               int r, int pass, int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    int Wn = ceil_div(W, n), Hn = ceil_div(H, n), hdi, vdj;
    prop_sources(pass & 3, &hdi, &vdj);
    for (int jj = 0; jj < Hn; ++jj) {
        int j = vdj < 0 ? jj : Hn - 1 - jj;
        for (int ii = 0; ii < Wn; ++ii) {
            int i = hdi < 0 ? ii : Wn - 1 - ii;
            int k = j * Wn + i, x = i * n, y = j * n;
            uint32_t bc = cost[k];
            int bfx = flow[2 * k], bfy = flow[2 * k + 1];
            for (int src = 0; src < 2; ++src) {  /* horizontal, then vertical source */
                int si = src == 0 ? i + hdi : i, sj = src == 0 ? j : j + vdj;
                if (si < 0 || si >= Wn || sj < 0 || sj >= Hn) continue;
                int ks = sj * Wn + si;
                if (cost[ks] == OR_UNSET) continue;
                int fx = flow[2 * ks], fy = flow[2 * ks + 1];
                if (bc != OR_UNSET && fx == bfx && fy == bfy) continue;
                if (!target_in(W, H, x, y, fx, fy, s)) continue;
                uint32_t e = E(Da, Db, W, H, m, r, x, y, fx, fy, s);
                *n_evals += 1;
                if (e < bc) { bc = e; bfx = fx; bfy = fy; }
            }
            cost[k] = bc;
            flow[2 * k] = (int16_t)bfx;
            flow[2 * k + 1] = (int16_t)bfy;
        }
    }
}

void or_propagate_raster(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int r, int pass,
                         int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    propagate_raster_g(cost_u8, 0, Da, Db, W, H, n, n, r, pass, flow, cost, n_evals);
}

/* SplitMix64 output mixer (Steele, Lea, Flood 2014). */
uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Counter of one random draw: direction stream, level, step, cell. */
uint64_t or_rs_counter(int stream, int level, int pass, int j, int i)
{
    return ((uint64_t)(stream & 0xFF) << 56) | ((uint64_t)(level & 0xFF) << 48) |
           ((uint64_t)(pass & 0xFFFF) << 32) | ((uint64_t)(j & 0xFFFF) << 16) | (uint64_t)(i & 0xFFFF);
}

/* Integer random-search offset of a cell, uniform on [-Rn, Rn]^2: the low
 * and high 32-bit halves of the draw are mapped to [0, 2Rn] by
 * multiply-shift. */
void or_rs_offset(uint64_t seed, int stream, int level, int pass, int j, int i, int Rn, int *ox, int *oy)
{
    uint64_t h = or_mix64(seed ^ or_mix64(or_rs_counter(stream, level, pass, j, i)));
    uint64_t span = (uint64_t)(2 * Rn + 1);
    *ox = (int)(((h & 0xFFFFFFFFULL) * span) >> 32) - Rn;
    *oy = (int)(((h >> 32) * span) >> 32) - Rn;
}

/* One random-search step (Sec. 3.1): every set cell tries its flow plus a
 * random offset and keeps it if E_n strictly decreases.  Offset (0, 0) and
 * targets outside the image are skipped. */
static void random_search_g(or_cost_fn E, int s, const void *Da, const void *Db, int W, int H, int n, int m, int r,
                            int Rn, uint64_t seed, int stream, int level, int pass, int16_t *flow, uint32_t *cost,
                            uint64_t *n_evals, int nthreads)
{
    int Wn = ceil_div(W, n), Hn = ceil_div(H, n);
    uint64_t cnt = 0;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for reduction(+ : cnt) schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int j = 0; j < Hn; ++j)
        for (int i = 0; i < Wn; ++i) {
            int k = j * Wn + i, x = i * n, y = j * n, ox, oy;
            if (cost[k] == OR_UNSET) continue;
            /* offsets uniform on [-Rn, Rn]^2 in units of 1/2^s pixel */
            or_rs_offset(seed, stream, level, pass, j, i, Rn * (1 << s), &ox, &oy);
            if (ox == 0 && oy == 0) continue;
            int fx = flow[2 * k] + ox, fy = flow[2 * k + 1] + oy;
            if (!target_in(W, H, x, y, fx, fy, s)) continue;
            uint32_t e = E(Da, Db, W, H, m, r, x, y, fx, fy, s);
            cnt += 1;
            if (e < cost[k]) {
                cost[k] = e;
                flow[2 * k] = (int16_t)fx;
                flow[2 * k + 1] = (int16_t)fy;
            }
        }
    *n_evals += cnt;
}

void or_random_search(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int r, int Rn,
                      uint64_t seed, int stream, int level, int pass, int16_t *flow, uint32_t *cost,
                      uint64_t *n_evals, int nthreads)
{
    random_search_g(cost_u8, 0, Da, Db, W, H, n, n, r, Rn, seed, stream, level, pass, flow, cost, n_evals, nthreads);
}

/* Forward-backward consistency (Sec. 3.7): keep pixel p of field a iff it is
 * set, its target q = p + F_a(p) is set in field b and
 * |F_a(p) + F_b(q)| < eps (exact integer test).  Flows in units of 1/2^s
 * pixel: q is the pixel nearest to the target (halves rounded up) and the
 * test is |F_a(p) + F_b(q)|^2 < (eps 2^s)^2 in those units. */
static void consistency_g(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb, int W,
                          int H, int s, double eps, uint8_t *keep)
{
    int S = 1 << s;
    double lim = eps * S;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t k = (size_t)y * W + x;
            keep[k] = 0;
            if (ca[k] == OR_UNSET) continue;
            int qx = (x * S + fa[2 * k] + S / 2) / S, qy = (y * S + fa[2 * k + 1] + S / 2) / S;
            size_t kq = (size_t)qy * W + qx;
            if (cb[kq] == OR_UNSET) continue;
            int64_t dx = fa[2 * k] + fb[2 * kq], dy = fa[2 * k + 1] + fb[2 * kq + 1];
            keep[k] = (double)(dx * dx + dy * dy) < lim * lim;
        }
}

void or_consistency(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb,
                    int W, int H, double eps, uint8_t *keep)
{
    consistency_g(fa, ca, fb, cb, W, H, 0, eps, keep);
}

/* The check on fields of the grid of scale n (Flow Fields+ Fast x2, Sec.
 * 3.4: one match per n x n region): cell (i, j) is pixel p = (i n, j n); the
 * backward match used for its target t = p + F_a is the one of the region
 * holding t, cell (floor(t.x / n), floor(t.y / n)); keep iff both are set
 * and |F_a + F_b|^2 < eps^2 (exact integers, compared in double).  n = 1
 * is or_consistency. */
void or_consistency_grid(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb, int W,
                         int H, int n, double eps, uint8_t *keep)
{
    int Wn = ceil_div(W, n), Hn = ceil_div(H, n);
    for (int j = 0; j < Hn; ++j)
        for (int i = 0; i < Wn; ++i) {
            size_t k = (size_t)j * Wn + i;
            keep[k] = 0;
            if (ca[k] == OR_UNSET) continue;
            int tx = i * n + fa[2 * k], ty = j * n + fa[2 * k + 1];
            if (tx < 0 || tx >= W || ty < 0 || ty >= H) continue;
            size_t kq = (size_t)(ty / n) * Wn + (size_t)(tx / n);
            if (cb[kq] == OR_UNSET) continue;
            int64_t dx = fa[2 * k] + fb[2 * kq], dy = fa[2 * k + 1] + fb[2 * kq + 1];
            keep[k] = (double)(dx * dx + dy * dy) < eps * eps;
        }
}

/* Consistency against two backward fields (Sec. 3.7): keep pixel p of
 * field a iff it passes the check of or_consistency against field b1 and
 * against field b2 (fields with different generator seeds and possibly
 * different patch radii); deleted if it fails either. */
void or_consistency2(const int16_t *fa, const uint32_t *ca, const int16_t *fb1, const uint32_t *cb1,
                     const int16_t *fb2, const uint32_t *cb2, int W, int H, double eps, uint8_t *keep)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t k = (size_t)y * W + x;
            keep[k] = 0;
            if (ca[k] == OR_UNSET) continue;
            int qx = x + fa[2 * k], qy = y + fa[2 * k + 1];
            size_t kq = (size_t)qy * W + qx;
            int ok = 1;
            const int16_t *fb[2] = {fb1, fb2};
            const uint32_t *cb[2] = {cb1, cb2};
            for (int j = 0; j < 2 && ok; ++j) {
                if (cb[j][kq] == OR_UNSET) {
                    ok = 0;
                    break;
                }
                int64_t dx = fa[2 * k] + fb[j][2 * kq], dy = fa[2 * k + 1] + fb[j][2 * kq + 1];
                ok = (double)(dx * dx + dy * dy) < eps * eps;
            }
            keep[k] = (uint8_t)ok;
        }
}

/* Region filter (Sec. 3.7, after the consistency check): the kept pixels
 * form regions, two 4-neighbours belonging to the same region iff their
 * flows differ by less than 3 px (|F(p) - F(q)|^2 < 9, exact).  A region of
 * fewer than s pixels is deleted if one of its pixels could take in, by the
 * same rule, a 4-neighbour that the consistency check removed (set, cost not
 * UNSET, but not kept).  keep_out = keep_in minus the deleted regions.
 * Breadth-first search over each region in turn. */
static int region_link(const int16_t *f, size_t a, size_t b)
{
    int dx = f[2 * a] - f[2 * b], dy = f[2 * a + 1] - f[2 * b + 1];
    return dx * dx + dy * dy < 9;
}

void or_region_filter(const int16_t *flow, const uint32_t *cost, const uint8_t *keep_in, int W, int H, int s,
                      uint8_t *keep_out)
{
    size_t N = (size_t)W * H;
    int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * N);
    size_t *queue = (size_t *)malloc(sizeof(size_t) * N);
    for (size_t k = 0; k < N; ++k) comp[k] = -1;
    memcpy(keep_out, keep_in, N);
    const int ddx[4] = {1, -1, 0, 0}, ddy[4] = {0, 0, 1, -1};
    for (size_t k0 = 0; k0 < N; ++k0) {
        if (!keep_in[k0] || comp[k0] >= 0) continue;
        size_t head = 0, tail = 0;
        queue[tail++] = k0;
        comp[k0] = (int32_t)k0;
        int touches = 0;
        while (head < tail) {
            size_t k = queue[head++];
            int x = (int)(k % W), y = (int)(k / W);
            for (int d = 0; d < 4; ++d) {
                int nx = x + ddx[d], ny = y + ddy[d];
                if (nx < 0 || nx >= W || ny < 0 || ny >= H) continue;
                size_t kn = (size_t)ny * W + nx;
                if (!region_link(flow, k, kn)) continue;
                if (keep_in[kn]) {
                    if (comp[kn] < 0) {
                        comp[kn] = (int32_t)k0;
                        queue[tail++] = kn;
                    }
                } else if (cost[kn] != OR_UNSET) {
                    touches = 1;  /* a removed outlier the region could take in */
                }
            }
        }
        if (tail < (size_t)s && touches)
            for (size_t i = 0; i < tail; ++i) keep_out[queue[i]] = 0;
    }
    free(comp);
    free(queue);
}

/* Sparsification (Sec. 3.8): in every q x q region of the filtered field a
 * (regions anchored at (0, 0), ragged at the right and bottom) that still
 * holds at least e kept samples, select the kept sample whose consistency
 * errors |F_a(p) + F_b1(p + F_a(p))| (+ the same against b2 when b2 is
 * given) sum to the least, in double precision; ties go to the smallest
 * row-major pixel index.  sel[region] = y * W + x of the selection, or -1.
 * A kept sample whose target leaves the image is not a candidate. */
void or_sparsify(const int16_t *fa, const uint8_t *keep, const int16_t *fb1, const int16_t *fb2, int W, int H,
                 int q, int e, int32_t *sel)
{
    int Wq = (W + q - 1) / q, Hq = (H + q - 1) / q;
    for (int ry = 0; ry < Hq; ++ry)
        for (int rx = 0; rx < Wq; ++rx) {
            int count = 0;
            int32_t best = -1;
            double best_err = 0.0;
            for (int y = ry * q; y < ry * q + q && y < H; ++y)
                for (int x = rx * q; x < rx * q + q && x < W; ++x) {
                    size_t k = (size_t)y * W + x;
                    if (!keep[k]) continue;
                    ++count;
                    int tx = x + fa[2 * k], ty = y + fa[2 * k + 1];
                    if (tx < 0 || tx >= W || ty < 0 || ty >= H) continue;
                    size_t kt = (size_t)ty * W + tx;
                    double dx = fa[2 * k] + fb1[2 * kt], dy = fa[2 * k + 1] + fb1[2 * kt + 1];
                    double err = sqrt(dx * dx + dy * dy);
                    if (fb2) {
                        double ex = fa[2 * k] + fb2[2 * kt], ey = fa[2 * k + 1] + fb2[2 * kt + 1];
                        err += sqrt(ex * ex + ey * ey);
                    }
                    if (best < 0 || err < best_err) {  /* row-major scan: ties keep the earlier */
                        best = (int32_t)k;
                        best_err = err;
                    }
                }
            sel[(size_t)ry * Wq + rx] = count >= e ? best : -1;
        }
}

/* R_n = floor(R * n) with R = R_num / R_den (R6). */
int or_rs_radius(int n, int R_num, int R_den) { return (int)(((int64_t)R_num * n) / R_den); }

/* The scales of the schedule, coarse to fine (Sec. 3.2): stage k has the
 * grid scale n (the cells p = (i n, j n) that propagate and search) and the
 * patch scale m (patch spacing, blur and random-search distance).  Without
 * sub-scales m = n for n = 2^(L-1), ..., 2^lmin.  With sub-scales (Sec.
 * 3.3, table of scales and sub-scales, R31) every scale n >= 2 below the
 * coarsest is preceded, on the same grid, by the sub-scale m = 3n/2: for
 * L = 4 the stages are (8,8) (4,6) (4,4) (2,3) (2,2) (1,1).  gen is the
 * generator's level field: log2 n, plus 16 on a sub-scale stage. */
typedef struct {
    int n, m, gen;
} or_stage;

int or_make_stages(int L, int lmin, int sub, int *stage_n, int *stage_m)
{
    int k = 0;
    for (int level = L - 1; level >= lmin; --level) {
        int n = 1 << level;
        if (sub && level < L - 1 && n >= 2) {
            stage_n[k] = n;
            stage_m[k] = 3 * n / 2;
            ++k;
        }
        stage_n[k] = n;
        stage_m[k] = n;
        ++k;
    }
    return k;
}

/* Steps of one stage.  The original schedule (Sec. 3.2): T propagation
 * steps, a random search at R_m after each but the last.  Flow Fields+
 * (Sec. 3.3): first P steps whose random searches use R_m^+ = R^+ m, then T
 * steps at R_m; random searches sit only between two steps of the same
 * group (P - 1 and T - 1 of them), and the step index t, which sets the
 * direction t mod 4 and keys the generator, runs on over both groups.
 * Flow Fields+ Fast (Sec. 3.4): the finest stage run runs only Tfine steps
 * at R_m (no R^+ group) when Tfine > 0. */
typedef struct {
    int P, T;      /* steps at R_m^+, then at R_m */
    int Rn, Rnp;   /* R_m and R_m^+ */
} or_scale_steps;

static or_scale_steps scale_steps(int m, int finest, int T, int R_num, int R_den, int P, int Rp_num, int Tfine)
{
    or_scale_steps st;
    st.P = P;
    st.T = T;
    if (finest && Tfine > 0) {
        st.P = 0;
        st.T = Tfine;
    }
    st.Rn = or_rs_radius(m, R_num, R_den);
    st.Rnp = or_rs_radius(m, Rp_num, R_den);
    return st;
}

/* Patch-scale change on one grid (the step from a sub-scale m = 3n/2 to the
 * scale n, Sec. 3.3): every set cell keeps its flow and evaluates its cost
 * at the new patch scale m. */
static void rescore_g(or_cost_fn E, int s, const void *Da, const void *Db, int W, int H, int n, int m, int r,
                      int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    int Wn = ceil_div(W, n), Hn = ceil_div(H, n);
    for (int j = 0; j < Hn; ++j)
        for (int i = 0; i < Wn; ++i) {
            int k = j * Wn + i;
            if (cost[k] == OR_UNSET) continue;
            cost[k] = E(Da, Db, W, H, m, r, i * n, j * n, flow[2 * k], flow[2 * k + 1], s);
            *n_evals += 1;
        }
}

void or_rescore(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int m, int r, int16_t *flow,
                uint32_t *cost, uint64_t *n_evals)
{
    rescore_g(cost_u8, 0, Da, Db, W, H, n, m, r, flow, cost, n_evals);
}

/* The steps with a patch scale m apart from the grid scale n (a sub-scale
 * stage); Da, Db: features of patch scale m. */
void or_seed_level_m(const int16_t *cflow, const uint32_t *ccost, const uint8_t *Da, const uint8_t *Db, int W, int H,
                     int n, int m, int r, int16_t *flow, uint32_t *cost, uint64_t *n_evals)
{
    seed_level_g(cost_u8, 0, cflow, ccost, Da, Db, W, H, n, m, r, flow, cost, n_evals);
}

void or_propagate_m(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int m, int r, int pass, int16_t *flow,
                    uint32_t *cost, uint64_t *n_evals, int nthreads)
{
    propagate_g(cost_u8, 0, Da, Db, W, H, n, m, r, pass, flow, cost, n_evals, nthreads);
}

void or_random_search_m(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int m, int r, int Rn,
                        uint64_t seed, int stream, int gen, int pass, int16_t *flow, uint32_t *cost,
                        uint64_t *n_evals, int nthreads)
{
    random_search_g(cost_u8, 0, Da, Db, W, H, n, m, r, Rn, seed, stream, gen, pass, flow, cost, n_evals, nthreads);
}

/* One direction of the multi-scale Flow Field (Sec. 3.2), a -> b, over the
 * stages of or_make_stages: Da[k], Db[k] are the features of patch scale
 * stage_m[k]; nn_l candidates per seed (Eq. 4); raster: serial-order
 * propagation steps instead of checkerboard ones; rstep = 2: the seeds are
 * taken from the even pixels only (Flow Fields+ Fast x2, Sec. 3.4).  The
 * result is the grid of the last stage. */
static void flow_one_direction(or_cost_fn E, int s, const uint8_t *Nq, const uint8_t *Nr, const void *const *Da,
                               const void *const *Db, int W, int H, int nst, const int *stage_n, const int *stage_m,
                               int T, int r, int R_num, int R_den, int P, int Rp_num, int Tfine, int nn_l, int raster,
                               int rstep, uint64_t seed, int stream, int nthreads, int16_t *flow_out,
                               uint32_t *cost_out, uint64_t *n_evals)
{
    int nc = stage_n[0];
    int Wc = ceil_div(W, nc), Hc = ceil_div(H, nc);
    size_t cells0 = (size_t)W * H;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)Wc * Hc * nn_l);
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)Wc * Hc * nn_l);
    int16_t *fl[2];
    uint32_t *co[2];
    for (int b = 0; b < 2; ++b) {
        fl[b] = (int16_t *)malloc(sizeof(int16_t) * 2 * cells0);
        co[b] = (uint32_t *)malloc(sizeof(uint32_t) * cells0);
    }
    if (nn_l == 1 && rstep == 1)
        or_nn(Nq, Nr, W, H, nc, idx, dist, nthreads);
    else
        or_nn_topl_step(Nq, Nr, W, H, nc, nn_l, rstep, idx, dist, nthreads);
    int cur = 0;
    init_coarse_g(E, s, idx, nn_l, Da[0], Db[0], W, H, nc, stage_m[0], r, fl[cur], co[cur], n_evals);
    for (int k = 0; k < nst; ++k) {
        int n = stage_n[k], m = stage_m[k];
        int level = 0;
        while ((1 << level) < n) ++level;
        int gen = level + (m != n ? 16 : 0);
        if (k > 0 && n == stage_n[k - 1]) {
            rescore_g(E, s, Da[k], Db[k], W, H, n, m, r, fl[cur], co[cur], n_evals);
        } else if (k > 0) {
            seed_level_g(E, s, fl[cur], co[cur], Da[k], Db[k], W, H, n, m, r, fl[cur ^ 1], co[cur ^ 1], n_evals);
            cur ^= 1;
        }
        or_scale_steps st = scale_steps(m, k == nst - 1, T, R_num, R_den, P, Rp_num, Tfine);
        for (int t = 0; t < st.P + st.T; ++t) {
            if (raster)
                propagate_raster_g(E, s, Da[k], Db[k], W, H, n, m, r, t, fl[cur], co[cur], n_evals);
            else
                propagate_g(E, s, Da[k], Db[k], W, H, n, m, r, t, fl[cur], co[cur], n_evals, nthreads);
            int last_of_group = t == st.P - 1 || t == st.P + st.T - 1;
            if (!last_of_group)
                random_search_g(E, s, Da[k], Db[k], W, H, n, m, r, t < st.P ? st.Rnp : st.Rn, seed, stream, gen, t,
                                fl[cur], co[cur], n_evals, nthreads);
        }
    }
    int nl = stage_n[nst - 1];
    size_t cells_out = (size_t)ceil_div(W, nl) * ceil_div(H, nl);
    memcpy(flow_out, fl[cur], sizeof(int16_t) * 2 * cells_out);
    memcpy(cost_out, co[cur], sizeof(uint32_t) * cells_out);
    for (int b = 0; b < 2; ++b) { free(fl[b]); free(co[b]); }
    free(idx);
    free(dist);
}

/* The whole hot path for one image pair: scale-space descriptors of both
 * images at every level, forward field (img1 -> img2, stream 0), backward
 * field (img2 -> img1, stream 1) and both consistency masks.
 * n_evals[0], n_evals[1]: number of E_n evaluations of each direction.
 * s > 0: the subpixel form (flows, random-search offsets and the
 * consistency threshold in units of 1/2^s pixel, costs of or_cost_sub).
 * nn_l in [1, 16]: seeds reranked among the nn_l nearest pixels (Eq. 4);
 * raster != 0: propagation steps in serial order (propagate_raster_g);
 * fast_x2 != 0: Flow Fields+ Fast x2 (Sec. 3.4), the fields and masks are
 * grids of scale 2 ([ceil(H/2)][ceil(W/2)]) checked by or_consistency_grid. */
static int flow_fields_g(const uint8_t *img1, const uint8_t *img2, int W, int H, int L, int T, int r, int R_num,
                         int R_den, int P, int Rp_num, int Tfine, int s, int nn_l, int raster, int fast_x2, int sub,
                         double eps, uint64_t seed, int nthreads,
                         int16_t *flow_fwd, int16_t *flow_bwd, uint32_t *cost_fwd, uint32_t *cost_bwd,
                         uint8_t *keep_fwd, uint8_t *keep_bwd, uint64_t *n_evals)
{
    if (W < 1 || H < 1 || W > 32767 || H > 32767 || L < 1 || L > 7 || T < 1 || r < 0 || r > 7 ||
        R_num < 0 || R_den < 1 || P < 0 || Rp_num < 0 || Tfine < 0 || P + T > 64 || Tfine > 64 || s < 0 || s > 3 ||
        (s > 0 && (W > (32767 >> s) || H > (32767 >> s))) || nn_l < 1 || nn_l > 16 || (fast_x2 && (L < 2 || s > 0)) ||
        (sub && fast_x2))
        return 1;
    size_t np = (size_t)W * H;
    uint8_t *blur = (uint8_t *)malloc(np);
    int stage_n[16], stage_m[16];
    int nst = or_make_stages(L, fast_x2 ? 1 : 0, sub, stage_n, stage_m);
    /* features of every stage's patch scale (level-1 ones for the NN seed) */
    uint8_t *D1[16], *D2[16], *N1 = (uint8_t *)malloc(np * 16), *N2 = (uint8_t *)malloc(np * 16);
    for (int k = 0; k <= nst; ++k) {
        int m = k < nst ? stage_m[k] : 1;
        uint8_t *a = k < nst ? (D1[k] = (uint8_t *)malloc(np * 16)) : N1;
        uint8_t *b = k < nst ? (D2[k] = (uint8_t *)malloc(np * 16)) : N2;
        or_blur(img1, W, H, m, blur);
        or_descriptor(blur, W, H, m, a);
        or_blur(img2, W, H, m, blur);
        or_descriptor(blur, W, H, m, b);
    }
    or_cost_fn E = s > 0 ? cost_u8_sub : cost_u8;
    n_evals[0] = n_evals[1] = 0;
    int rstep = fast_x2 ? 2 : 1;
    flow_one_direction(E, s, N1, N2, (const void *const *)D1, (const void *const *)D2, W, H, nst, stage_n, stage_m,
                       T, r, R_num, R_den, P, Rp_num, Tfine, nn_l, raster, rstep, seed, 0, nthreads, flow_fwd,
                       cost_fwd, &n_evals[0]);
    flow_one_direction(E, s, N2, N1, (const void *const *)D2, (const void *const *)D1, W, H, nst, stage_n, stage_m,
                       T, r, R_num, R_den, P, Rp_num, Tfine, nn_l, raster, rstep, seed, 1, nthreads, flow_bwd,
                       cost_bwd, &n_evals[1]);
    if (fast_x2) {
        or_consistency_grid(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, 2, eps, keep_fwd);
        if (keep_bwd) or_consistency_grid(flow_bwd, cost_bwd, flow_fwd, cost_fwd, W, H, 2, eps, keep_bwd);
    } else {
        consistency_g(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, s, eps, keep_fwd);
        if (keep_bwd) consistency_g(flow_bwd, cost_bwd, flow_fwd, cost_fwd, W, H, s, eps, keep_bwd);
    }
    for (int k = 0; k < nst; ++k) { free(D1[k]); free(D2[k]); }
    free(N1);
    free(N2);
    free(blur);
    return 0;
}

int or_flow_fields(const uint8_t *img1, const uint8_t *img2, int W, int H, int L, int T, int r,
                   int R_num, int R_den, int P, int Rp_num, int Tfine, double eps, uint64_t seed, int nthreads,
                   int16_t *flow_fwd, int16_t *flow_bwd, uint32_t *cost_fwd, uint32_t *cost_bwd,
                   uint8_t *keep_fwd, uint8_t *keep_bwd, uint64_t *n_evals)
{
    return flow_fields_g(img1, img2, W, H, L, T, r, R_num, R_den, P, Rp_num, Tfine, 0, 1, 0, 0, 0, eps, seed, nthreads,
                         flow_fwd, flow_bwd, cost_fwd, cost_bwd, keep_fwd, keep_bwd, n_evals);
}

/* or_flow_fields with every option: subpixel form s, nn_l seed candidates,
 * serial-order (raster) propagation, Flow Fields+ Fast x2 (fast_x2; outputs
 * on the grid of scale 2), sub-scales (sub; Sec. 3.3). */
int or_flow_fields_x(const uint8_t *img1, const uint8_t *img2, int W, int H, int L, int T, int r, int R_num,
                     int R_den, int P, int Rp_num, int Tfine, int s, int nn_l, int raster, int fast_x2, int sub,
                     double eps, uint64_t seed, int nthreads, int16_t *flow_fwd, int16_t *flow_bwd,
                     uint32_t *cost_fwd, uint32_t *cost_bwd, uint8_t *keep_fwd, uint8_t *keep_bwd, uint64_t *n_evals)
{
    return flow_fields_g(img1, img2, W, H, L, T, r, R_num, R_den, P, Rp_num, Tfine, s, nn_l, raster, fast_x2, sub,
                         eps, seed, nthreads, flow_fwd, flow_bwd, cost_fwd, cost_bwd, keep_fwd, keep_bwd, n_evals);
}

/* The subpixel form of or_flow_fields (flows in units of 1/2^s pixel). */
int or_flow_fields_sub(const uint8_t *img1, const uint8_t *img2, int W, int H, int L, int T, int r, int R_num,
                       int R_den, int P, int Rp_num, int Tfine, int s, double eps, uint64_t seed, int nthreads,
                       int16_t *flow_fwd, int16_t *flow_bwd, uint32_t *cost_fwd, uint32_t *cost_bwd,
                       uint8_t *keep_fwd, uint8_t *keep_bwd, uint64_t *n_evals)
{
    return flow_fields_g(img1, img2, W, H, L, T, r, R_num, R_den, P, Rp_num, Tfine, s, 1, 0, 0, 0, eps, seed, nthreads,
                         flow_fwd, flow_bwd, cost_fwd, cost_bwd, keep_fwd, keep_bwd, n_evals);
}

/* One propagation step and one random-search step of the subpixel form
 * (flows in units of 1/2^s pixel; Rn in pixels). */
void or_propagate_sub(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int r, int s, int pass,
                      int16_t *flow, uint32_t *cost, uint64_t *n_evals, int nthreads)
{
    propagate_g(cost_u8_sub, s, Da, Db, W, H, n, n, r, pass, flow, cost, n_evals, nthreads);
}

void or_random_search_sub(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int r, int s, int Rn,
                          uint64_t seed, int stream, int level, int pass, int16_t *flow, uint32_t *cost,
                          uint64_t *n_evals, int nthreads)
{
    random_search_g(cost_u8_sub, s, Da, Db, W, H, n, n, r, Rn, seed, stream, level, pass, flow, cost, n_evals,
                    nthreads);
}

void or_consistency_sub(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb, int W, int H,
                        int s, double eps, uint8_t *keep)
{
    consistency_g(fa, ca, fb, cb, W, H, s, eps, keep);
}

/* The same multi-scale schedule on learned float features: F1[l], F2[l] are
 * the 16-channel float32 feature maps of scale 2^l of both images; the NN
 * seed runs on their level-1 maps quantised to bytes (or_quantize_u8), the
 * matching error is or_cost_f32 (costs are returned as float bit patterns).
 */
int or_flow_fields_f32(const float *const *F1, const float *const *F2, int W, int H, int L, int T, int r,
                       int R_num, int R_den, int P, int Rp_num, int Tfine, double eps, uint64_t seed,
                       int nthreads, int16_t *flow_fwd, int16_t *flow_bwd, uint32_t *cost_fwd, uint32_t *cost_bwd,
                       uint8_t *keep_fwd, uint8_t *keep_bwd, uint64_t *n_evals)
{
    if (W < 1 || H < 1 || W > 32767 || H > 32767 || L < 1 || L > 7 || T < 1 || r < 0 || r > 7 ||
        R_num < 0 || R_den < 1 || P < 0 || Rp_num < 0 || Tfine < 0 || P + T > 64 || Tfine > 64)
        return 1;
    size_t np = (size_t)W * H;
    uint8_t *q1 = (uint8_t *)malloc(np * 16), *q2 = (uint8_t *)malloc(np * 16);
    or_quantize_pair_u8(F1[0], F2[0], (int64_t)np * 16, q1, q2);
    n_evals[0] = n_evals[1] = 0;
    int stage_n[16], stage_m[16];
    int nst = or_make_stages(L, 0, 0, stage_n, stage_m);
    const float *S1[16], *S2[16];  /* stage k is scale 2^(L-1-k) */
    for (int k = 0; k < nst; ++k) {
        S1[k] = F1[L - 1 - k];
        S2[k] = F2[L - 1 - k];
    }
    flow_one_direction(cost_f32, 0, q1, q2, (const void *const *)S1, (const void *const *)S2, W, H, nst, stage_n,
                       stage_m, T, r, R_num, R_den, P, Rp_num, Tfine, 1, 0, 1, seed, 0, nthreads, flow_fwd, cost_fwd,
                       &n_evals[0]);
    flow_one_direction(cost_f32, 0, q2, q1, (const void *const *)S2, (const void *const *)S1, W, H, nst, stage_n,
                       stage_m, T, r, R_num, R_den, P, Rp_num, Tfine, 1, 0, 1, seed, 1, nthreads, flow_bwd, cost_bwd,
                       &n_evals[1]);
    or_consistency(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, eps, keep_fwd);
    if (keep_bwd) or_consistency(flow_bwd, cost_bwd, flow_fwd, cost_fwd, W, H, eps, keep_bwd);
    free(q1);
    free(q2);
    return 0;
}
