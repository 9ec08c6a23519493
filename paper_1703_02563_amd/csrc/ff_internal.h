// Host-side interface between the C ABI (ff_api.hip) and the kernel
// translation units.  Every launcher enqueues on `stream` and returns the
// launch status; none allocates or synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ffh {

constexpr int kMaxJobs = 16;   // descriptor jobs per launch: 2 images x 7 levels (+ slack)
constexpr int kMaxDirs = 2;    // forward and backward field in one launch

// One scale-space descriptor job: image -> blurred -> descriptors at scale n.
struct DescJob {
  const uint8_t *img;
  uint16_t *hsum;
  uint8_t *blurred;
  uint8_t *desc;     // padded, phase-ordered map (see desc_index); nullable: only the copies below
  uint8_t *compact;  // nullable: row-major [H][W][16] copy (the NN seed's input)
  uint8_t *wform;    // nullable: weight-class row map (see wform_index)
  int n;
};
struct DescJobs {
  DescJob job[kMaxJobs];
  int count;
  int W, H;
};
hipError_t launch_descriptors(const DescJobs &jobs, hipStream_t stream);

// Fills `count` 64-bit words with `value`.
hipError_t launch_fill_u64(uint64_t *dst, uint64_t value, int64_t count, hipStream_t stream);

// Brute-force NN of the coarsest grid on int8 matrix cores.
struct NNDir {
  const uint8_t *Dq;   // level-1 descriptors of the image holding the query cells
  const uint8_t *Dr;   // level-1 descriptors of the reference image
  int32_t *nb;         // per-reference squared norm of (d - 128), padded to a multiple of 32
  uint64_t *keys;      // per-query packed result (see ff_nn.hip)
};
struct NNArgs {
  NNDir dir[kMaxDirs];
  int ndir;
  int W, H, nc, Wc, M, N;
  int chunk_tiles;  // reference tiles (32 each) per workgroup; set by launch_nn
};
hipError_t launch_nn(const NNArgs &args, hipStream_t stream);

// The l nearest references of every query (1 <= l <= kTopLMax), after
// launch_nn: l - 1 more passes of the NN kernel, pass k leaving out the
// references up to pass k-1's key (see ff_nn.hip).
constexpr int kTopLMax = 8;
struct TopLDir {
  const uint8_t *Dq;       // level-1 row-major descriptors of the query image
  const uint8_t *Dr;       // the same of the reference image
  const int32_t *nb;       // reference norms of launch_nn
  const uint64_t *nn_key;  // launch_nn's keys (pass 0)
  uint64_t *keys;          // [kTopLMax - 1][M] scratch: keys of passes 1 ..
  uint64_t *cand;          // [M][l] output: (squared distance << 32) | q, ranked; ~0 past N
};
struct TopLArgs {
  TopLDir dir[kMaxDirs];
  int ndir, l;
  int W, H, nc, Wc, M, N;
  int even_refs;  // 1: the references are the even-pixel subset (launch_gather_even)
};
struct TopLPrev {
  const uint64_t *key[kMaxDirs];
};
size_t topl_scratch_bytes(int M);  // the keys of passes 1 .. kTopLMax - 1 of one direction
// Flow Fields+ Fast x2: the level-1 descriptors of the pixels with even x
// and y ([ceil(H/2)][ceil(W/2)][16], the NN's references), and the NN keys
// over that subset turned into keys naming image pixels.
hipError_t launch_gather_even(const uint8_t *desc1, uint8_t *out, int W, int H, hipStream_t stream);
hipError_t launch_remap_even(uint64_t *keys, int M, int W, hipStream_t stream);
hipError_t launch_topl(const TopLArgs &args, hipStream_t stream);

// Launch tables of the temporally blocked level kernels, per scale log2 n
// (the C ABI's ff_tuning): kernel variant and most propagation steps per
// launch (0: as many as the window's halo allows), for the byte descriptors
// and for the learned float features.  Passed with every call; the library
// keeps only the immutable default.
constexpr int kTuneScales = 7;
struct Tuning {
  int variant[kTuneScales];
  int passes[kTuneScales];
  int variant_f32[kTuneScales];
  int passes_f32[kTuneScales];
};
const Tuning &default_tuning();
bool tuning_ok(const Tuning &t);

// Per-direction state of a level grid.
struct LevelDir {
  const void *Da;      // scale-n descriptors (or float features) of the source image
  const void *Db;      // scale-n descriptors (or float features) of the target image
  int32_t *flow;       // packed (dx, dy) int16 pairs, [cells]
  uint32_t *cost;      // [cells]
  const int32_t *cflow;   // coarser grid (seeding only)
  const uint32_t *ccost;
  const uint64_t *nn_key; // coarsest init only
  const uint8_t *Dq1;     // level-1 descriptors of the source image (coarsest init only)
  unsigned long long *n_evals;
  unsigned long long *n_work;  // nullable [2]: evaluations computed (all of them count in both entries here)
  int stream_id;
};
struct LevelArgs {
  LevelDir dir[kMaxDirs];
  int ndir;
  int fcost;  // 0: byte descriptors, SAD; 1: float32 16-channel features, SSD; 2: byte descriptors, 1/8-px flows
  int W, H, n, Wn, Hn, radius;
  int ns;     // patch scale of a sub-scale stage (patch p + ns (u, v), features of scale ns); 0: n
  int Rn, level, pass;
  uint64_t seed;
};
hipError_t launch_init_coarse(const LevelArgs &a, hipStream_t stream);
hipError_t launch_seed_level(const LevelArgs &a, hipStream_t stream);
hipError_t launch_propagate(const LevelArgs &a, hipStream_t stream);  // both half-sweeps
hipError_t launch_random_search(const LevelArgs &a, hipStream_t stream);
// Seed rerank (Eq. 1, Eq. 4) at the coarsest scale: per cell the candidate
// of cand[dir] ([cells][l], launch_topl's output) with the lowest E_nc, the
// earlier rank on equal cost, written to nn_key in launch_nn's format for
// the initialisation; counts every candidate but the winner (the
// initialisation evaluates the winner again).
hipError_t launch_rerank(const LevelArgs &a, const uint64_t *const *cand, int l, hipStream_t stream);
// One propagation step in serial order (anti-diagonal wavefronts over tiles;
// integer costs only).
hipError_t launch_propagate_raster(const LevelArgs &a, hipStream_t stream);
// Patch-scale change on one grid (sub-scales): every set cell's cost at
// patch scale a.ns, with a.ns's features in Da/Db.
hipError_t launch_rescore(const LevelArgs &a, hipStream_t stream);

// Temporally blocked run of propagation / random-search steps of one scale
// (patch radius 3).  Passes [t_begin, t_end) of T; a random-search step
// follows pass t iff t is neither P - 1 nor T - 1, with radius Rnp for t < P
// and Rn after (Flow Fields+ groups).  halo[] = half-sweeps reading the left,
// right, top, bottom side over the run (at most kLevelHalo each).
constexpr int kLevelHalo = 6;
constexpr int kLevelContinue = 0;  // state from the level grid in global memory
constexpr int kLevelInit = 1;      // coarsest scale: flows from the NN keys
constexpr int kLevelSeed = 2;      // seeds from the coarser grid, other cells UNSET
struct LevelKDir {
  const uint8_t *Da;
  const uint8_t *Db;
  const uint8_t *Wa;  // weight-class row maps of the two images (nullable: the
  const uint8_t *Wb;  //   variants that use them fall back to descriptor quads)
  int32_t *flow;            // written: the owned cells after the run
  uint32_t *cost;
  const int32_t *flow_in;   // read by a continuing run (never the buffer it writes:
  const uint32_t *cost_in;  // other workgroups of the launch write theirs meanwhile)
  const int32_t *cflow;
  const uint32_t *ccost;
  const uint64_t *nn_key;
  unsigned long long *n_evals;
  // nullable [2]: [0] evaluations computed for owned cells, [1] all
  // evaluations computed, halo recomputation included (n_evals counts the
  // unblocked schedule's evaluations, some of which a consistent state makes
  // unnecessary)
  unsigned long long *n_work;
  int stream_id;
};
struct LevelKArgs {
  LevelKDir dir[kMaxDirs];
  int ndir;
  int W, H, n, Wn, Hn, level, Rn;
  int Rnp, P;  // the first P steps' random searches use Rnp (Flow Fields+); 0: none
  uint64_t seed;
  int t_begin, t_end, T;  // T: steps of the scale; no random search after steps P - 1 and T - 1
  int mode;
  int fcost;    // 0: byte descriptor maps; 1: padded float feature maps (64-byte entries)
  int variant;  // the launch table's variant of this scale (byte or float table by fcost)
  int radius;   // patch radius: 3, or 2 and 4 (byte descriptors only); 0 means 3
  int tiles_x;  // set by launch_level
  int halo[4];
  int sub_m;    // a sub-scale stage's patch scale m (Da/Db: image-order maps of scale m, radius 3); 0: n
};
// Padded, phase-ordered copy of a float [H][W][16] feature map of scale n.
hipError_t launch_pad_features(const float *f, int W, int H, int n, float *out, hipStream_t stream);
hipError_t launch_level(LevelKArgs a, hipStream_t stream);
// per-scale launchers of the blocked kernels (ff_level_s<log2n>.hip)
struct BatchStage;
#define FF_LEVEL_SCALE_DECL(k)                                                                          \
  hipError_t launch_level_scale##k(const LevelKArgs &a, const BatchStage *batch, int variant, hipStream_t s); \
  hipError_t launch_level_f32_scale##k(const LevelKArgs &a, int variant, hipStream_t s); \
  hipError_t launch_level_r2_scale##k(const LevelKArgs &a, int variant, hipStream_t s); \
  hipError_t launch_level_r4_scale##k(const LevelKArgs &a, int variant, hipStream_t s);
FF_LEVEL_SCALE_DECL(0)
FF_LEVEL_SCALE_DECL(1)
FF_LEVEL_SCALE_DECL(2)
FF_LEVEL_SCALE_DECL(3)
FF_LEVEL_SCALE_DECL(4)
FF_LEVEL_SCALE_DECL(5)
FF_LEVEL_SCALE_DECL(6)
#undef FF_LEVEL_SCALE_DECL
int level_window_halo(int variant);              // window halo of a byte-descriptor variant
int level_window_halo_f32(int variant);          // the same for a float-feature variant
bool level_map_fits(int W, int H, int log2n);  // scale-n map under 2^31 bytes (quad evaluations)
bool level_uses_wform(int variant);  // the variant evaluates interior cells on weight-class row maps
void level_halo(int t_begin, int t_end, int halo[4]);
int level_variant_count();      // byte-descriptor variants + the step-wise schedule
int level_variant_count_f32();
bool level_stepwise(int variant);  // the variant index that selects the step-wise schedule
// The blocked kernels run this patch radius at these sizes (radius 3; radii
// 2 and 4 with descriptor maps inside the 32-bit offsets of the quad
// evaluations).
bool level_blocked_ok(int W, int H, int L, int radius);

// ---- batches of pairs of different sizes (one launch per stage) ----------
constexpr int kMaxBatch = 256;
constexpr int kMaxScales = 7;

// Device-side record of one pair of a batch: inputs, outputs and the pair's
// share of the workspace (all device pointers).
struct BatchPair {
  const uint8_t *img[2];
  int W, H;
  uint16_t *hsum[2][kMaxScales];
  uint8_t *blur[2][kMaxScales];
  uint8_t *desc[2][kMaxScales];  // padded maps
  uint8_t *wform[2][kMaxScales]; // weight-class row maps
  uint8_t *desc1[2];             // row-major scale-1 descriptors (NN seed)
  int32_t *nb[2];
  uint64_t *keys[2];
  int32_t *gflow[kMaxScales][2];
  uint32_t *gcost[kMaxScales][2];
  int32_t *sflow[kMaxScales][2];  // second buffer of each level grid (runs alternate)
  uint32_t *scost[kMaxScales][2];
  uint8_t *keep[2];
  unsigned long long *evals;  // [2]
};

// Work items of one stage: pair p owns items [prefix[p], prefix[p+1]).
struct BatchStage {
  const BatchPair *pairs;
  int npairs, total;
  int L, n, lv;  // scales of the schedule, scale of this stage
  int src, dst;  // level stages: grid buffer read (continuing runs) and written, 0 = gflow/gcost, 1 = sflow/scost
  int prefix[kMaxBatch + 1];
};
hipError_t launch_batch_descriptors(const BatchStage &rows, hipStream_t stream);
hipError_t launch_batch_nn(const BatchStage &norms, const BatchStage &fill, const BatchStage &nn, hipStream_t stream);
hipError_t launch_batch_level(const LevelKArgs &base, const BatchStage &tiles, bool maps_fit, hipStream_t stream);
hipError_t launch_batch_consistency(const BatchStage &rows, float eps, hipStream_t stream);
// items per pair of each stage (host)
int batch_nn_items(int W, int H, int L);
// tiles of one direction for the kernel that runs at that scale (the current
// variant, or its fallback when a map does not fit the quad addressing)
int level_tiles(int Wn, int Hn, int variant, bool maps_fit);

// Float patch cost of 16-channel float32 feature maps (learned data term).
struct CostArgs {
  const float *f1;       // [H][W][16]
  const float *f2;       // [H][W][16]
  const int4 *entries;   // [count] = (x, y, fx, fy)
  int count;
  int W, H, n, radius;
  float *cost;            // forward output [count]
  const float *grad_cost; // backward input [count]
  int64_t *acc1, *acc2;   // backward fixed-point accumulators [H][W][16] (acc2 = acc1 + H*W*16)
  int64_t *overflow;      // one word after acc2: count of terms or sums that left the fixed-point range
  float *grad_f1, *grad_f2;
};
hipError_t launch_cost_fwd(const CostArgs &a, hipStream_t stream);
hipError_t launch_cost_bwd(const CostArgs &a, hipStream_t stream);

// 3x3 convolution, NHWC bf16 activations, weights [cout][9][cin] bf16.
struct ConvArgs {
  const uint16_t *in;  // [B][H][W][cin] bf16
  const uint16_t *w;   // [cout][9][cin] bf16
  const float *bias;   // [cout] (nullable)
  int B, H, W, cin, cout, relu;
  float *out_f32;      // [B][H][W][cout] (nullable)
  uint16_t *out_bf16;  // [B][H][W][cout] (nullable)
  const float *gout;   // weight gradient: upstream gradient [B][H][W][cout] f32
  float *partial;      // weight gradient: per-block partial sums
};
hipError_t launch_conv_fwd(const ConvArgs &a, hipStream_t stream);
// The descriptor network 1 -> 32 -> 32 -> 16 for inference in one launch.
struct NetArgs {
  const uint16_t *in;             // [B][H][W] bf16 network input
  const uint16_t *w1, *w2, *w3;   // bf16 [32][9][1], [32][9][32], [16][9][32]
  const float *b1, *b2, *b3;      // [32], [32], [16]
  int B, H, W, normalize;
  float delta;
  float *out;                     // [B][H][W][16]
};
hipError_t launch_descnet_fwd(const NetArgs &a, hipStream_t stream);
hipError_t launch_weight_flip(const uint16_t *w, uint16_t *wf, int cin, int cout, hipStream_t stream);
int wgrad_blocks(int B, int H);
hipError_t launch_wgrad(const ConvArgs &a, float *gw, float *gbias, hipStream_t stream);
hipError_t launch_relu_bwd(const uint16_t *act, const float *g, float *gout, uint16_t *gout_bf16, long long count,
                           hipStream_t stream);
hipError_t launch_f32_to_bf16(const float *x, uint16_t *y, long long count, hipStream_t stream);
hipError_t launch_image_to_bf16(const uint8_t *img, uint16_t *out, long long count, hipStream_t stream);
hipError_t launch_triplet_hinge(const float *cost, int m, float margin, float scale, float weight, float *grad,
                                float *loss, hipStream_t stream);
hipError_t launch_l2norm16_fwd(const float *f, long long P, float delta, float *y, float *inv_norm,
                               hipStream_t stream);
hipError_t launch_l2norm16_bwd(const float *y, const float *inv_norm, const float *g, long long P, float *gin,
                               hipStream_t stream);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int count, float lr, float b1, float b2,
                       float eps, int step, uint16_t *p_bf16, hipStream_t stream);
hipError_t launch_quantize(const float *f, long long count, float *part, uint8_t *q, hipStream_t stream);
hipError_t launch_quantize_pair(const float *f1, const float *f2, long long count, float *part, uint8_t *q1,
                                uint8_t *q2, hipStream_t stream);
size_t quantize_scratch_bytes();  // float scratch of launch_quantize and launch_quantize_pair

// Consistency of field a against field b (full resolution).
size_t region_filter_scratch_bytes(int W, int H);
hipError_t launch_region_filter(const int16_t *flow, const uint32_t *cost, const uint8_t *keep, int W, int H, int s,
                                void *work, uint8_t *keep_out, hipStream_t stream);
// The same with the library's static per-device scratch (W * H at most
// region_filter_noalloc_max_pixels()).
size_t region_filter_noalloc_max_pixels();
hipError_t launch_region_filter_noalloc(const int16_t *flow, const uint32_t *cost, const uint8_t *keep, int W, int H,
                                        int s, uint8_t *keep_out, hipStream_t stream);
hipError_t launch_sparsify(const int16_t *fa, const uint8_t *keep, const int16_t *fb1, const int16_t *fb2, int W,
                           int H, int q, int e, int32_t *sel, hipStream_t stream);
hipError_t launch_consistency2(const int16_t *fa, const uint32_t *ca, const int16_t *fb1, const uint32_t *cb1,
                               const int16_t *fb2, const uint32_t *cb2, int W, int H, float eps, uint8_t *keep,
                               hipStream_t stream);
// Fields on the grid of scale n, one match per n x n region (Fast x2).
hipError_t launch_consistency_grid(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb,
                                  int W, int H, int n, float eps, uint8_t *keep_a, uint8_t *keep_b,
                                  hipStream_t stream);
// sb: flows in units of 1/2^sb pixel (0: whole pixels)
hipError_t launch_consistency(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb,
                              int W, int H, float eps, uint8_t *keep_a, uint8_t *keep_b, hipStream_t stream,
                              int sb = 0);

}  // namespace ffh
