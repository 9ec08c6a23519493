// C ABI of the Flow Fields hot path (declared in include/flowfields.h):
// argument validation, workspace carving and the per-level schedule of
// Sec. 3.2 (coarsest NN seed, then per scale: seeding, T propagation steps
// with T-1 random-search steps in between), forward and backward fields
// enqueued together, then the consistency check of Sec. 3.7.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/flowfields.h"
#include "ff_device.h"
#include "ff_internal.h"

namespace {

constexpr int kMaxLevels = 7;

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }
inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
inline bool is_pow2(int n) { return n >= 1 && n <= 64 && (n & (n - 1)) == 0; }
inline bool dims_ok(int W, int H) { return W >= 1 && H >= 1 && W <= 32767 && H <= 32767; }
// The NN seed addresses the level-1 descriptors (16 bytes a pixel) with
// 32-bit offsets: fewer than 2^27 pixels per image.
inline bool nn_dims_ok(int W, int H) { return dims_ok(W, H) && (long long)W * H < (1ll << 27); }

ff_status from_hip(hipError_t e) { return e == hipSuccess ? FF_OK : FF_ERR_LAUNCH; }

// The call's launch tables (ff_tuning and ffh::Tuning have the same fields).
ffh::Tuning tuning_of(const ff_tuning *t) {
  if (!t) return ffh::default_tuning();
  ffh::Tuning u;
  for (int k = 0; k < ffh::kTuneScales; ++k) {
    u.variant[k] = t->variant[k];
    u.passes[k] = t->passes[k];
    u.variant_f32[k] = t->variant_f32[k];
    u.passes_f32[k] = t->passes_f32[k];
  }
  return u;
}

bool params_ok(const ff_params *p) {
  return p && p->levels >= 1 && p->levels <= kMaxLevels && p->iters >= 1 && p->iters <= 64 && p->radius >= 0 &&
         p->radius <= 7 && p->R_num >= 0 && p->R_den >= 1 && p->R_num <= 1 << 20 && p->R_den <= 1 << 20 &&
         p->plus_iters >= 0 && p->plus_iters + p->iters <= 64 && p->Rp_num >= 0 && p->Rp_num <= 1 << 20 &&
         p->fine_iters >= 0 && p->fine_iters <= 64 && (p->subpixel == 0 || p->subpixel == 3) && p->nn_l >= 0 &&
         p->nn_l <= ffh::kTopLMax && (p->raster == 0 || p->raster == 1) && (p->fast_x2 == 0 || p->fast_x2 == 1) &&
         (!p->fast_x2 || (p->levels >= 2 && p->subpixel == 0)) && (p->subscales == 0 || p->subscales == 1) &&
         !(p->subscales && p->fast_x2) && ffh::tuning_ok(tuning_of(p->tuning));
}

// Seed candidates of the call (0 and 1: the exact NN alone).
int nn_l_of(const ff_params *p) { return p->nn_l > 1 ? p->nn_l : 1; }

// Subpixel flows (1/8 px in int16) reach at most 4095 px.
bool sub_dims_ok(const ff_params *p, int W, int H) {
  return p->subpixel == 0 || (W <= (32767 >> p->subpixel) && H <= (32767 >> p->subpixel));
}

int rs_radius(int n, int R_num, int R_den) { return (int)(((int64_t)R_num * n) / R_den); }

// The sub-scale stage before scale n = 2^lv (Sec. 3.3): patch scale 3n/2.
int subscale_of(int lv) { return 3 << (lv - 1); }

// Stages of the sub-scale schedule, coarse to fine: (grid scale n, patch
// scale m); every scale n >= 2 below the coarsest is preceded by (n, 3n/2).
int subscale_stages(int L, int *stage_lv, int *stage_m) {
  int k = 0;
  for (int lv = L - 1; lv >= 0; --lv) {
    if (lv < L - 1 && lv >= 1) {
      stage_lv[k] = lv;
      stage_m[k++] = subscale_of(lv);
    }
    stage_lv[k] = lv;
    stage_m[k++] = 1 << lv;
  }
  return k;
}

// Steps of scale lv: P steps whose random searches use R_n^+, then T at R_n
// (Flow Fields+, Sec. 3.3; P = 0 is the original schedule of Sec. 3.2), or
// only fine_iters steps at R_n on the finest scale (Flow Fields+ Fast, Sec.
// 3.4).  A random search follows step t unless t ends its group.
struct ScaleSteps {
  int P, T, Rn, Rnp;
  int total() const { return P + T; }
  bool rs_after(int t) const { return t != P - 1 && t != P + T - 1; }
  int radius(int t) const { return t < P ? Rnp : Rn; }
};

ScaleSteps scale_steps(const ff_params *p, int lv) {
  const int n = 1 << lv;
  ScaleSteps st{p->plus_iters, p->iters, rs_radius(n, p->R_num, p->R_den), rs_radius(n, p->Rp_num, p->R_den)};
  if (lv == (p->fast_x2 ? 1 : 0) && p->fine_iters > 0) {  // the finest scale run
    st.P = 0;
    st.T = p->fine_iters;
  }
  return st;
}

// Device workspace of ff_flow_fields, carved in this order.
struct Layout {
  size_t hsum, blur, desc[2][kMaxLevels], wform[2][kMaxLevels], sdesc[2][kMaxLevels], desc1, desc1e, nb, keys, topl,
      cand, grids, sgrids, evals, total;
  size_t N, Npad, M;
  int L;
};

// Bytes of a padded scale-n descriptor map (replicated border of 3n pixels).
size_t desc_map_bytes(int W, int H, int n) {
  const size_t P = (size_t)ffk::desc_pad(n);
  return (W + 2 * P) * (H + 2 * P) * 16;
}

Layout layout(int W, int H, const ff_params *p) {
  Layout l{};
  l.L = p->levels;
  l.N = (size_t)W * H;
  l.Npad = (l.N + 31) & ~(size_t)31;
  const int nc = 1 << (p->levels - 1);
  l.M = (size_t)ceil_div(W, nc) * ceil_div(H, nc);
  size_t off = 0;
  l.hsum = off; off = align256(off + 2 * l.L * l.N * sizeof(uint16_t));
  l.blur = off; off = align256(off + 2 * l.L * l.N);
  for (int im = 0; im < 2; ++im)
    for (int lv = 0; lv < l.L; ++lv) {
      l.desc[im][lv] = off;
      off = align256(off + desc_map_bytes(W, H, 1 << lv));
    }
  for (int im = 0; im < 2; ++im)
    for (int lv = 0; lv < l.L; ++lv) {
      l.wform[im][lv] = off;
      off = align256(off + ffk::wform_bytes(W, H, 1 << lv));
    }
  // sub-scales: the maps of patch scale 3n/2 for the scales n = 2^lv, 1 <= lv <= L - 2
  for (int im = 0; im < 2; ++im)
    for (int lv = 1; lv + 1 < l.L; ++lv) {
      l.sdesc[im][lv] = off;
      if (p->subscales) off = align256(off + desc_map_bytes(W, H, subscale_of(lv)));
    }
  l.desc1 = off; off = align256(off + 2 * l.N * 16);
  // Fast x2: the NN's references, the even pixels of both images
  l.desc1e = off;
  if (p->fast_x2) off = align256(off + 2 * (size_t)ceil_div(W, 2) * ceil_div(H, 2) * 16);
  l.nb = off; off = align256(off + 2 * l.Npad * sizeof(int32_t));
  l.keys = off; off = align256(off + 2 * l.M * sizeof(uint64_t));
  // seed rerank: bound, collection and ranked candidates of both directions
  l.topl = off;
  if (p->nn_l > 1) off = align256(off + 2 * ffh::topl_scratch_bytes((int)l.M));
  l.cand = off;
  if (p->nn_l > 1) off = align256(off + 2 * l.M * p->nn_l * sizeof(uint64_t));
  l.grids = off;
  for (int lv = 1; lv < l.L; ++lv) {
    const size_t cells = (size_t)ceil_div(W, 1 << lv) * ceil_div(H, 1 << lv);
    off = align256(off + 2 * cells * 2 * sizeof(uint32_t));
  }
  l.sgrids = off;
  for (int lv = 0; lv < l.L; ++lv) {
    const size_t cells = (size_t)ceil_div(W, 1 << lv) * ceil_div(H, 1 << lv);
    off = align256(off + 2 * cells * 2 * sizeof(uint32_t));
  }
  l.evals = off; off = align256(off + 2 * sizeof(uint64_t));
  l.total = off;
  return l;
}

// Second buffers of the level grids (flow then cost per direction), carved
// from `base + off` for scales 0..L-1.
void carve_second_grids(char *base, size_t off, int W, int H, int L, int32_t *sflow[][2], uint32_t *scost[][2]) {
  for (int lv = 0; lv < L; ++lv) {
    const size_t cells = (size_t)ceil_div(W, 1 << lv) * ceil_div(H, 1 << lv);
    for (int dr = 0; dr < 2; ++dr) {
      sflow[lv][dr] = reinterpret_cast<int32_t *>(base + off) + (size_t)dr * 2 * cells;
      scost[lv][dr] = reinterpret_cast<uint32_t *>(sflow[lv][dr] + cells);
    }
    off = align256(off + 2 * cells * 2 * sizeof(uint32_t));
  }
}

ffh::LevelArgs one_dir_args(const uint8_t *Da, const uint8_t *Db, int W, int H, int n, int radius, int16_t *flow,
                            uint32_t *cost, uint64_t *n_evals) {
  ffh::LevelArgs a{};
  a.ndir = 1;
  a.W = W;
  a.H = H;
  a.n = n;
  a.Wn = ceil_div(W, n);
  a.Hn = ceil_div(H, n);
  a.radius = radius;
  a.dir[0].Da = Da;
  a.dir[0].Db = Db;
  a.dir[0].flow = reinterpret_cast<int32_t *>(flow);
  a.dir[0].cost = cost;
  a.dir[0].n_evals = reinterpret_cast<unsigned long long *>(n_evals);
  return a;
}

// End of the longest run of passes starting at t0 whose halo fits the level
// kernel's window (halo cells per side), at most maxp passes (maxp <= 0: no
// limit).
int run_end(int t0, int T, int maxp, int halo = ffh::kLevelHalo) {
  int t1 = t0 + 1, h[4];
  while (t1 < T && (maxp <= 0 || t1 - t0 < maxp)) {
    ffh::level_halo(t0, t1 + 1, h);
    if (h[0] > halo || h[1] > halo || h[2] > halo || h[3] > halo) break;
    ++t1;
  }
  return t1;
}

// Runs of passes of one scale: [t0, t1) pairs; the number of launches.
int level_runs(const ffh::Tuning &tun, int lv, int T, int fcost, int runs[][2]) {
  int m = 0, t0 = 0;
  const int halo = fcost ? ffh::level_window_halo_f32(tun.variant_f32[lv]) : ffh::level_window_halo(tun.variant[lv]);
  const int maxp = fcost ? tun.passes_f32[lv] : tun.passes[lv];
  while (t0 < T) {
    const int t1 = run_end(t0, T, maxp, halo);
    runs[m][0] = t0;
    runs[m][1] = t1;
    ++m;
    t0 = t1;
  }
  return m;
}

// The passes of one scale as temporally blocked launches: each launch runs
// the longest run of passes whose halo fits the kernel's window (and the
// run-length table).  k.dir[] must hold the per-direction pointers, flow/cost
// being the level grid that receives the result; the scale fields are set
// here.  A continuing launch reads the grid the previous launch wrote and
// writes the other one (sflow/scost: one more grid per direction, needed
// only when the scale takes more than one launch), so that no workgroup
// reads cells another workgroup of the same launch is writing; the last
// launch writes flow/cost.
hipError_t run_level_blocked(ffh::LevelKArgs k, int W, int H, int lv, const ff_params *p, int first_mode,
                             hipStream_t s, int32_t *const *sflow = nullptr, uint32_t *const *scost = nullptr,
                             int sub_m = 0) {
  const int n = 1 << lv;
  // a sub-scale stage (patch scale sub_m, Sec. 3.3) runs the Flow Fields+
  // step groups at the random-search distances of its patch scale; its
  // generator level field is lv + 16 (as in the per-step kernels)
  const ScaleSteps sst = sub_m ? ScaleSteps{p->plus_iters, p->iters, rs_radius(sub_m, p->R_num, p->R_den),
                                            rs_radius(sub_m, p->Rp_num, p->R_den)}
                               : scale_steps(p, lv);
  const int T = sst.total();
  k.W = W;
  k.H = H;
  k.n = n;
  k.Wn = ceil_div(W, n);
  k.Hn = ceil_div(H, n);
  k.level = lv + (sub_m ? 16 : 0);
  k.sub_m = sub_m;
  k.Rn = sst.Rn;
  k.Rnp = sst.Rnp;
  k.P = sst.P;
  k.seed = p->seed;
  k.T = T;
  k.radius = p->radius;
  const ffh::Tuning tun = tuning_of(p->tuning);
  k.variant = k.fcost ? tun.variant_f32[lv] : tun.variant[lv];
  int runs[64][2];
  const int m = level_runs(tun, lv, T, k.fcost, runs);
  const bool two = m > 1 || first_mode == ffh::kLevelContinue;
  if (two && (!sflow || !scost)) return hipErrorInvalidValue;
  int32_t *main_f[ffh::kMaxDirs];
  uint32_t *main_c[ffh::kMaxDirs];
  for (int dr = 0; dr < k.ndir; ++dr) {
    main_f[dr] = k.dir[dr].flow;
    main_c[dr] = k.dir[dr].cost;
  }
  for (int r = 0; r < m; ++r) {
    const bool to_main = ((m - 1 - r) & 1) == 0;  // the last launch writes the level grid
    for (int dr = 0; dr < k.ndir; ++dr) {
      if (r > 0 || first_mode == ffh::kLevelContinue) {
        // a continuing run reads what the previous run wrote (the caller's
        // state for a first continuing run: it sits in flow/cost and is
        // copied to the second buffer below when the first run writes there)
        k.dir[dr].flow_in = r > 0 ? k.dir[dr].flow : main_f[dr];
        k.dir[dr].cost_in = r > 0 ? k.dir[dr].cost : main_c[dr];
      }
      k.dir[dr].flow = to_main ? main_f[dr] : sflow[dr];
      k.dir[dr].cost = to_main ? main_c[dr] : scost[dr];
    }
    if (r == 0 && first_mode == ffh::kLevelContinue && to_main) {
      // the first continuing run would read and write the caller's grid:
      // move the input to the second buffer first
      const size_t cells = (size_t)k.Wn * k.Hn;
      for (int dr = 0; dr < k.ndir; ++dr) {
        hipError_t e = hipMemcpyAsync(sflow[dr], main_f[dr], cells * 4, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(scost[dr], main_c[dr], cells * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        k.dir[dr].flow_in = sflow[dr];
        k.dir[dr].cost_in = scost[dr];
      }
    }
    ffh::level_halo(runs[r][0], runs[r][1], k.halo);
    k.t_begin = runs[r][0];
    k.t_end = runs[r][1];
    k.mode = r > 0 ? ffh::kLevelContinue : first_mode;
    hipError_t e = ffh::launch_level(k, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The passes of one scale with one launch per step over all cells: the
// coarsest scale's NN initialisation or the seeding from the coarser scale,
// then T propagation passes (two half-sweeps each) with T-1 random searches.
// a.dir[] must hold the per-direction pointers; the scale fields are set here.
hipError_t run_level_steps(ffh::LevelArgs a, int W, int H, int lv, int L, const ff_params *p, hipStream_t s) {
  const int n = 1 << lv;
  a.W = W;
  a.H = H;
  a.n = n;
  a.Wn = ceil_div(W, n);
  a.Hn = ceil_div(H, n);
  a.level = lv;
  const ScaleSteps st = scale_steps(p, lv);
  a.Rn = st.Rn;
  a.radius = p->radius;
  a.seed = p->seed;
  hipError_t e = (lv == L - 1) ? ffh::launch_init_coarse(a, s) : ffh::launch_seed_level(a, s);
  if (e != hipSuccess) return e;
  for (int t = 0; t < st.total(); ++t) {
    a.pass = t;
    e = p->raster ? ffh::launch_propagate_raster(a, s) : ffh::launch_propagate(a, s);
    if (e != hipSuccess) return e;
    a.Rn = st.radius(t);
    if (st.rs_after(t) && (e = ffh::launch_random_search(a, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// One stage of the sub-scale schedule with one launch per step: grid scale
// 2^lv, patch scale m (a.dir[].Da/Db: the features of scale m); entry 0:
// the coarsest stage's NN initialisation, 1: the same grid at a new patch
// scale (costs re-evaluated), 2: the hand-over from the coarser grid.  The
// generator's level field is lv, plus 16 on a sub-scale stage.
hipError_t run_stage(ffh::LevelArgs a, int W, int H, int lv, int m, int entry, bool finest, const ff_params *p,
                     hipStream_t s) {
  const int n = 1 << lv;
  a.W = W;
  a.H = H;
  a.n = n;
  a.ns = m;
  a.Wn = ceil_div(W, n);
  a.Hn = ceil_div(H, n);
  a.level = lv + (m != n ? 16 : 0);
  a.radius = p->radius;
  a.seed = p->seed;
  ScaleSteps st{p->plus_iters, p->iters, rs_radius(m, p->R_num, p->R_den), rs_radius(m, p->Rp_num, p->R_den)};
  if (finest && p->fine_iters > 0) {
    st.P = 0;
    st.T = p->fine_iters;
  }
  hipError_t e = entry == 0   ? ffh::launch_init_coarse(a, s)
                 : entry == 1 ? ffh::launch_rescore(a, s)
                              : ffh::launch_seed_level(a, s);
  if (e != hipSuccess) return e;
  for (int t = 0; t < st.total(); ++t) {
    a.pass = t;
    a.Rn = st.radius(t);
    e = p->raster ? ffh::launch_propagate_raster(a, s) : ffh::launch_propagate(a, s);
    if (e != hipSuccess) return e;
    if (st.rs_after(t) && (e = ffh::launch_random_search(a, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int ff_version(void) { return 1; }

const char *ff_status_str(ff_status s) {
  switch (s) {
    case FF_OK: return "ok";
    case FF_ERR_ARG: return "invalid argument";
    case FF_ERR_LAUNCH: return "kernel launch failed";
    case FF_ERR_WORKSPACE: return "workspace too small";
    case FF_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

size_t ff_descriptor_map_bytes(int32_t W, int32_t H, int32_t n) {
  if (!dims_ok(W, H) || n < 1 || n > 64) return 0;
  return desc_map_bytes(W, H, n);
}

size_t ff_wform_map_bytes(int32_t W, int32_t H, int32_t n) {
  if (!dims_ok(W, H) || n < 1 || n > 64) return 0;
  return ffk::wform_bytes(W, H, n);
}

ff_status ff_descriptors(const uint8_t *img, int32_t W, int32_t H, int32_t n, uint16_t *hsum, uint8_t *blurred,
                         uint8_t *desc, uint8_t *desc_rowmajor, uint8_t *wform, void *stream) {
  if (!img || !hsum || !blurred || !desc || !dims_ok(W, H) || n < 1 || n > 64) return FF_ERR_ARG;
  ffh::DescJobs jobs{};
  jobs.W = W;
  jobs.H = H;
  jobs.count = 1;
  jobs.job[0] = {img, hsum, blurred, desc, desc_rowmajor, wform, n};
  return from_hip(ffh::launch_descriptors(jobs, (hipStream_t)stream));
}

ff_status ff_init_nn(const uint8_t *desc_a1, const uint8_t *desc_b1, const uint8_t *desc_ac, const uint8_t *desc_bc,
                     int32_t W, int32_t H, int32_t nc, int32_t radius, int32_t *nb_scratch, uint64_t *nn_key,
                     int16_t *flow, uint32_t *cost, uint64_t *n_evals, void *stream) {
  if (!desc_a1 || !desc_b1 || !desc_ac || !desc_bc || !nb_scratch || !nn_key || !flow || !cost || !nn_dims_ok(W, H) ||
      !is_pow2(nc) || radius < 0 || radius > 7)
    return FF_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  ffh::NNArgs nn{};
  nn.ndir = 1;
  nn.W = W;
  nn.H = H;
  nn.nc = nc;
  nn.Wc = ceil_div(W, nc);
  nn.M = nn.Wc * ceil_div(H, nc);
  nn.N = W * H;
  nn.dir[0] = {desc_a1, desc_b1, nb_scratch, nn_key};
  hipError_t e = ffh::launch_nn(nn, s);
  if (e != hipSuccess) return FF_ERR_LAUNCH;
  ffh::LevelArgs a = one_dir_args(desc_ac, desc_bc, W, H, nc, radius, flow, cost, n_evals);
  a.dir[0].nn_key = nn_key;
  a.dir[0].Dq1 = desc_a1;
  return from_hip(ffh::launch_init_coarse(a, s));
}

size_t ff_nn_topl_scratch_bytes(int32_t W, int32_t H, int32_t nc) {
  if (!nn_dims_ok(W, H) || !is_pow2(nc) || nc > (1 << (kMaxLevels - 1))) return 0;
  const size_t M = (size_t)ceil_div(W, nc) * ceil_div(H, nc);
  return align256(M * sizeof(uint64_t)) + ffh::topl_scratch_bytes((int)M) +
         align256(M * ffh::kTopLMax * sizeof(uint64_t));
}

// The NN keys, then the l ranked candidates of every cell (scratch: keys,
// the top-l pass's parts, and -- when cand is NULL -- the candidates).
static hipError_t nn_topl_run(const uint8_t *desc_a1, const uint8_t *desc_b1, int W, int H, int nc, int l,
                              int32_t *nb_scratch, char *scratch, uint64_t *keys, uint64_t *cand, hipStream_t s) {
  ffh::NNArgs nn{};
  nn.ndir = 1;
  nn.W = W;
  nn.H = H;
  nn.nc = nc;
  nn.Wc = ceil_div(W, nc);
  nn.M = nn.Wc * ceil_div(H, nc);
  nn.N = W * H;
  nn.dir[0] = {desc_a1, desc_b1, nb_scratch, keys};
  hipError_t e = ffh::launch_nn(nn, s);
  if (e != hipSuccess) return e;
  ffh::TopLArgs tl{};
  tl.ndir = 1;
  tl.l = l;
  tl.W = W;
  tl.H = H;
  tl.nc = nc;
  tl.Wc = nn.Wc;
  tl.M = nn.M;
  tl.N = nn.N;
  ffh::TopLDir &d = tl.dir[0];
  d.Dq = desc_a1;
  d.Dr = desc_b1;
  d.nb = nb_scratch;
  d.nn_key = keys;
  d.keys = reinterpret_cast<uint64_t *>(scratch + align256((size_t)nn.M * sizeof(uint64_t)));
  d.cand = cand;
  return ffh::launch_topl(tl, s);
}

ff_status ff_nn_topl(const uint8_t *desc_a1, const uint8_t *desc_b1, int32_t W, int32_t H, int32_t nc, int32_t l,
                     int32_t *nb_scratch, void *scratch, size_t scratch_bytes, uint64_t *cand, void *stream) {
  if (!desc_a1 || !desc_b1 || !nb_scratch || !cand || !nn_dims_ok(W, H) || !is_pow2(nc) ||
      nc > (1 << (kMaxLevels - 1)) || l < 1 || l > ffh::kTopLMax)
    return FF_ERR_ARG;
  if (!scratch || scratch_bytes < ff_nn_topl_scratch_bytes(W, H, nc)) return FF_ERR_WORKSPACE;
  char *sp = static_cast<char *>(scratch);
  return from_hip(nn_topl_run(desc_a1, desc_b1, W, H, nc, l, nb_scratch, sp, reinterpret_cast<uint64_t *>(sp), cand,
                              (hipStream_t)stream));
}

ff_status ff_init_nn_l(const uint8_t *desc_a1, const uint8_t *desc_b1, const uint8_t *desc_ac, const uint8_t *desc_bc,
                       int32_t W, int32_t H, int32_t nc, int32_t radius, int32_t nn_l, int32_t *nb_scratch,
                       void *scratch, size_t scratch_bytes, uint64_t *nn_key, int16_t *flow, uint32_t *cost,
                       uint64_t *n_evals, void *stream) {
  if (nn_l < 0 || nn_l > ffh::kTopLMax) return FF_ERR_ARG;
  if (nn_l <= 1)
    return ff_init_nn(desc_a1, desc_b1, desc_ac, desc_bc, W, H, nc, radius, nb_scratch, nn_key, flow, cost, n_evals,
                      stream);
  if (!desc_a1 || !desc_b1 || !desc_ac || !desc_bc || !nb_scratch || !nn_key || !flow || !cost || !nn_dims_ok(W, H) ||
      !is_pow2(nc) || nc > (1 << (kMaxLevels - 1)) || radius < 0 || radius > 7)
    return FF_ERR_ARG;
  if (!scratch || scratch_bytes < ff_nn_topl_scratch_bytes(W, H, nc)) return FF_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char *sp = static_cast<char *>(scratch);
  const int M = ceil_div(W, nc) * ceil_div(H, nc);
  uint64_t *cand =
      reinterpret_cast<uint64_t *>(sp + align256((size_t)M * sizeof(uint64_t)) + ffh::topl_scratch_bytes(M));
  hipError_t e = nn_topl_run(desc_a1, desc_b1, W, H, nc, nn_l, nb_scratch, sp, nn_key, cand, s);
  if (e != hipSuccess) return FF_ERR_LAUNCH;
  ffh::LevelArgs a = one_dir_args(desc_ac, desc_bc, W, H, nc, radius, flow, cost, n_evals);
  a.dir[0].nn_key = nn_key;
  a.dir[0].Dq1 = desc_a1;
  const uint64_t *cands[1] = {cand};
  if ((e = ffh::launch_rerank(a, cands, nn_l, s)) != hipSuccess) return FF_ERR_LAUNCH;
  return from_hip(ffh::launch_init_coarse(a, s));
}

ff_status ff_seed_level(const int16_t *coarse_flow, const uint32_t *coarse_cost, const uint8_t *desc_a,
                        const uint8_t *desc_b, int32_t W, int32_t H, int32_t n, int32_t radius, int16_t *flow,
                        uint32_t *cost, uint64_t *n_evals, void *stream) {
  if (!coarse_flow || !coarse_cost || !desc_a || !desc_b || !flow || !cost || !dims_ok(W, H) || !is_pow2(n) ||
      n > 32 || radius < 0 || radius > 7)
    return FF_ERR_ARG;
  ffh::LevelArgs a = one_dir_args(desc_a, desc_b, W, H, n, radius, flow, cost, n_evals);
  a.dir[0].cflow = reinterpret_cast<const int32_t *>(coarse_flow);
  a.dir[0].ccost = coarse_cost;
  return from_hip(ffh::launch_seed_level(a, (hipStream_t)stream));
}

ff_status ff_propagate_level(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n,
                             int32_t radius, int32_t pass, int16_t *flow, uint32_t *cost, uint64_t *n_evals,
                             void *stream) {
  if (!desc_a || !desc_b || !flow || !cost || !dims_ok(W, H) || !is_pow2(n) || radius < 0 || radius > 7 ||
      pass < 0 || pass > 0xFFFF)
    return FF_ERR_ARG;
  ffh::LevelArgs a = one_dir_args(desc_a, desc_b, W, H, n, radius, flow, cost, n_evals);
  a.pass = pass;
  return from_hip(ffh::launch_propagate(a, (hipStream_t)stream));
}

ff_status ff_propagate_raster(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n,
                              int32_t radius, int32_t pass, int16_t *flow, uint32_t *cost, uint64_t *n_evals,
                              void *stream) {
  if (!desc_a || !desc_b || !flow || !cost || !dims_ok(W, H) || !is_pow2(n) || radius < 0 || radius > 7 ||
      pass < 0 || pass > 0xFFFF)
    return FF_ERR_ARG;
  ffh::LevelArgs a = one_dir_args(desc_a, desc_b, W, H, n, radius, flow, cost, n_evals);
  a.pass = pass;
  return from_hip(ffh::launch_propagate_raster(a, (hipStream_t)stream));
}

ff_status ff_rescore_level(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n, int32_t m,
                           int32_t radius, const int16_t *flow, uint32_t *cost, uint64_t *n_evals, void *stream) {
  if (!desc_a || !desc_b || !flow || !cost || !dims_ok(W, H) || !is_pow2(n) || m < 1 || m > 64 || radius < 0 ||
      radius > 7)
    return FF_ERR_ARG;
  ffh::LevelArgs a = one_dir_args(desc_a, desc_b, W, H, n, radius, const_cast<int16_t *>(flow), cost, n_evals);
  a.ns = m;
  return from_hip(ffh::launch_rescore(a, (hipStream_t)stream));
}

ff_status ff_random_search(const uint8_t *desc_a, const uint8_t *desc_b, int32_t W, int32_t H, int32_t n,
                           int32_t radius, int32_t Rn, uint64_t seed, int32_t stream_id, int32_t level, int32_t pass,
                           int16_t *flow, uint32_t *cost, uint64_t *n_evals, void *stream) {
  if (!desc_a || !desc_b || !flow || !cost || !dims_ok(W, H) || !is_pow2(n) || radius < 0 || radius > 7 ||
      Rn < 0 || Rn > 32767 || pass < 0 || pass > 0xFFFF || level < 0 || level > 0xFF || stream_id < 0 ||
      stream_id > 0xFF)
    return FF_ERR_ARG;
  ffh::LevelArgs a = one_dir_args(desc_a, desc_b, W, H, n, radius, flow, cost, n_evals);
  a.Rn = Rn;
  a.seed = seed;
  a.level = level;
  a.pass = pass;
  a.dir[0].stream_id = stream_id;
  return from_hip(ffh::launch_random_search(a, (hipStream_t)stream));
}

ff_status ff_consistency_filter(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b,
                                const uint32_t *cost_b, int32_t W, int32_t H, float eps, uint8_t *keep_a,
                                uint8_t *keep_b, void *stream) {
  if (!flow_a || !cost_a || !flow_b || !cost_b || !keep_a || !dims_ok(W, H) || !(eps >= 0.0f)) return FF_ERR_ARG;
  return from_hip(ffh::launch_consistency(flow_a, cost_a, flow_b, cost_b, W, H, eps, keep_a, keep_b,
                                          (hipStream_t)stream));
}

ff_status ff_consistency_filter_sub(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b,
                                    const uint32_t *cost_b, int32_t W, int32_t H, int32_t subpixel, float eps,
                                    uint8_t *keep_a, uint8_t *keep_b, void *stream) {
  if (!flow_a || !cost_a || !flow_b || !cost_b || !keep_a || !dims_ok(W, H) || !(eps >= 0.0f) || subpixel < 0 ||
      subpixel > 3)
    return FF_ERR_ARG;
  return from_hip(ffh::launch_consistency(flow_a, cost_a, flow_b, cost_b, W, H, eps, keep_a, keep_b,
                                          (hipStream_t)stream, subpixel));
}

ff_status ff_consistency_filter_grid(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b,
                                     const uint32_t *cost_b, int32_t W, int32_t H, int32_t n, float eps,
                                     uint8_t *keep_a, uint8_t *keep_b, void *stream) {
  if (!flow_a || !cost_a || !flow_b || !cost_b || !keep_a || !dims_ok(W, H) || !is_pow2(n) || !(eps >= 0.0f))
    return FF_ERR_ARG;
  return from_hip(ffh::launch_consistency_grid(flow_a, cost_a, flow_b, cost_b, W, H, n, eps, keep_a, keep_b,
                                               (hipStream_t)stream));
}

ff_status ff_consistency_filter2(const int16_t *flow_a, const uint32_t *cost_a, const int16_t *flow_b1,
                                 const uint32_t *cost_b1, const int16_t *flow_b2, const uint32_t *cost_b2, int32_t W,
                                 int32_t H, float eps, uint8_t *keep_a, void *stream) {
  if (!flow_a || !cost_a || !flow_b1 || !cost_b1 || !flow_b2 || !cost_b2 || !keep_a || !dims_ok(W, H) ||
      !(eps >= 0.0f))
    return FF_ERR_ARG;
  return from_hip(ffh::launch_consistency2(flow_a, cost_a, flow_b1, cost_b1, flow_b2, cost_b2, W, H, eps, keep_a,
                                           (hipStream_t)stream));
}

size_t ff_region_filter_scratch_bytes(int32_t W, int32_t H) {
  return dims_ok(W, H) ? ffh::region_filter_scratch_bytes(W, H) : 0;
}

ff_status ff_region_filter(const int16_t *flow, const uint32_t *cost, const uint8_t *keep_in, int32_t W, int32_t H,
                           int32_t s, void *scratch, size_t scratch_bytes, uint8_t *keep_out, void *stream) {
  if (!flow || !cost || !keep_in || !keep_out || !dims_ok(W, H) || s < 0 || keep_in == keep_out) return FF_ERR_ARG;
  if (!scratch || scratch_bytes < ffh::region_filter_scratch_bytes(W, H)) return FF_ERR_WORKSPACE;
  if ((uintptr_t)scratch & 3) return FF_ERR_ARG;  // 32-bit atomics on the parents and counters
  return from_hip(ffh::launch_region_filter(flow, cost, keep_in, W, H, s, scratch, keep_out, (hipStream_t)stream));
}

size_t ff_region_filter_noalloc_max_pixels(void) { return ffh::region_filter_noalloc_max_pixels(); }

ff_status ff_region_filter_noalloc(const int16_t *flow, const uint32_t *cost, const uint8_t *keep_in, int32_t W,
                                   int32_t H, int32_t s, uint8_t *keep_out, void *stream) {
  if (!flow || !cost || !keep_in || !keep_out || !dims_ok(W, H) || s < 0 || keep_in == keep_out) return FF_ERR_ARG;
  if ((size_t)W * H > ffh::region_filter_noalloc_max_pixels()) return FF_ERR_WORKSPACE;
  return from_hip(ffh::launch_region_filter_noalloc(flow, cost, keep_in, W, H, s, keep_out, (hipStream_t)stream));
}

ff_status ff_sparsify(const int16_t *flow_a, const uint8_t *keep_a, const int16_t *flow_b1, const int16_t *flow_b2,
                      int32_t W, int32_t H, int32_t q, int32_t e, int32_t *sel, void *stream) {
  if (!flow_a || !keep_a || !flow_b1 || !sel || !dims_ok(W, H) || q < 1 || q > 64 || e < 0) return FF_ERR_ARG;
  return from_hip(ffh::launch_sparsify(flow_a, keep_a, flow_b1, flow_b2, W, H, q, e, sel, (hipStream_t)stream));
}

size_t ff_run_level_scratch_bytes(int32_t W, int32_t H, int32_t level) {
  if (!dims_ok(W, H) || level < 0 || level >= kMaxLevels) return 0;
  return (size_t)ceil_div(W, 1 << level) * ceil_div(H, 1 << level) * 2 * sizeof(uint32_t);
}

ff_status ff_run_level(const uint8_t *desc_a, const uint8_t *desc_b, const uint8_t *wform_a, const uint8_t *wform_b,
                       int32_t W, int32_t H, int32_t level,
                       const ff_params *params, int32_t stream_id, int32_t mode, const uint64_t *nn_key,
                       const int16_t *coarse_flow, const uint32_t *coarse_cost, int16_t *flow, uint32_t *cost,
                       void *scratch, size_t scratch_bytes, uint64_t *n_evals, uint64_t *n_work, void *stream) {
  if (!desc_a || !desc_b || !flow || !cost || !dims_ok(W, H) || !params_ok(params) || level < 0 ||
      level >= kMaxLevels || stream_id < 0 || stream_id > 0xFF || mode < 0 || mode > 2 || (mode == 1 && !nn_key) ||
      (mode == 2 && (!coarse_flow || !coarse_cost)))
    return FF_ERR_ARG;
  if (!scratch || scratch_bytes < ff_run_level_scratch_bytes(W, H, level)) return FF_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (!sub_dims_ok(params, W, H)) return FF_ERR_ARG;
  if (params->subscales) return FF_ERR_UNSUPPORTED;  // a stage is not a scale: ff_flow_fields runs them
  const int n = 1 << level, r = params->radius;
  const ScaleSteps st = scale_steps(params, level);
  if (params->subpixel == 0 && !params->raster && ffh::level_blocked_ok(W, H, level + 1, r)) {
    ffh::LevelKArgs k{};
    k.ndir = 1;
    k.dir[0].Da = desc_a;
    k.dir[0].Db = desc_b;
    k.dir[0].Wa = wform_a;
    k.dir[0].Wb = wform_b;
    k.dir[0].flow = reinterpret_cast<int32_t *>(flow);
    k.dir[0].cost = cost;
    k.dir[0].nn_key = nn_key;
    k.dir[0].cflow = reinterpret_cast<const int32_t *>(coarse_flow);
    k.dir[0].ccost = coarse_cost;
    k.dir[0].n_evals = reinterpret_cast<unsigned long long *>(n_evals);
    k.dir[0].n_work = reinterpret_cast<unsigned long long *>(n_work);
    k.dir[0].stream_id = stream_id;
    const int first = mode == 1 ? ffh::kLevelInit : (mode == 2 ? ffh::kLevelSeed : ffh::kLevelContinue);
    int32_t *sf[1] = {static_cast<int32_t *>(scratch)};
    uint32_t *sc[1] = {reinterpret_cast<uint32_t *>(sf[0] + (size_t)ceil_div(W, n) * ceil_div(H, n))};
    return from_hip(run_level_blocked(k, W, H, level, params, first, s, sf, sc));
  }
  ffh::LevelArgs a = one_dir_args(desc_a, desc_b, W, H, n, r, flow, cost, n_evals);
  a.fcost = params->subpixel ? 2 : 0;
  a.level = level;
  a.seed = params->seed;
  a.Rn = st.Rn;
  a.dir[0].stream_id = stream_id;
  a.dir[0].nn_key = nn_key;
  a.dir[0].cflow = reinterpret_cast<const int32_t *>(coarse_flow);
  a.dir[0].ccost = coarse_cost;
  a.dir[0].n_work = reinterpret_cast<unsigned long long *>(n_work);
  hipError_t e = hipSuccess;
  if (mode == 1) return FF_ERR_UNSUPPORTED;  // the per-step path seeds through ff_init_nn
  if (mode == 2) e = ffh::launch_seed_level(a, s);
  for (int t = 0; t < st.total() && e == hipSuccess; ++t) {
    a.pass = t;
    e = params->raster ? ffh::launch_propagate_raster(a, s) : ffh::launch_propagate(a, s);
    a.Rn = st.radius(t);
    if (e == hipSuccess && st.rs_after(t)) e = ffh::launch_random_search(a, s);
  }
  return from_hip(e);
}

ff_status ff_run_level_pair(const uint8_t *desc_a, const uint8_t *desc_b, const uint8_t *wform_a,
                            const uint8_t *wform_b, int32_t W, int32_t H, int32_t level, const ff_params *params,
                            int32_t mode, const uint64_t *const *nn_key, const int16_t *const *coarse_flow,
                            const uint32_t *const *coarse_cost, int16_t *const *flow, uint32_t *const *cost,
                            void *scratch, size_t scratch_bytes, uint64_t *n_evals, uint64_t *n_work, void *stream) {
  if (!desc_a || !desc_b || !flow || !cost || !dims_ok(W, H) || !params_ok(params) || level < 0 ||
      level >= kMaxLevels || mode < 0 || mode > 2 || (mode == 1 && !nn_key) ||
      (mode == 2 && (!coarse_flow || !coarse_cost)) || !sub_dims_ok(params, W, H))
    return FF_ERR_ARG;
  for (int dr = 0; dr < 2; ++dr)
    if (!flow[dr] || !cost[dr] || (mode == 1 && !nn_key[dr]) ||
        (mode == 2 && (!coarse_flow[dr] || !coarse_cost[dr])))
      return FF_ERR_ARG;
  const size_t one = ff_run_level_scratch_bytes(W, H, level);
  if (!scratch || scratch_bytes < 2 * one) return FF_ERR_WORKSPACE;
  if (params->subpixel || params->raster || params->subscales || !ffh::level_blocked_ok(W, H, level + 1, params->radius))
    return FF_ERR_UNSUPPORTED;  // both directions in one launch: the blocked kernels only
  const int n = 1 << level;
  const size_t cells = (size_t)ceil_div(W, n) * ceil_div(H, n);
  const uint8_t *D[2] = {desc_a, desc_b}, *Wf[2] = {wform_a, wform_b};
  ffh::LevelKArgs k{};
  k.ndir = 2;
  int32_t *sf[2];
  uint32_t *sc[2];
  for (int dr = 0; dr < 2; ++dr) {
    ffh::LevelKDir &d = k.dir[dr];
    d.Da = D[dr];
    d.Db = D[dr ^ 1];
    d.Wa = Wf[dr];
    d.Wb = Wf[dr ^ 1];
    d.flow = reinterpret_cast<int32_t *>(flow[dr]);
    d.cost = cost[dr];
    d.nn_key = mode == 1 ? nn_key[dr] : nullptr;
    d.cflow = mode == 2 ? reinterpret_cast<const int32_t *>(coarse_flow[dr]) : nullptr;
    d.ccost = mode == 2 ? coarse_cost[dr] : nullptr;
    d.n_evals = n_evals ? reinterpret_cast<unsigned long long *>(n_evals + dr) : nullptr;
    d.n_work = reinterpret_cast<unsigned long long *>(n_work);
    d.stream_id = dr;
    sf[dr] = static_cast<int32_t *>(scratch) + (size_t)dr * 2 * cells;
    sc[dr] = reinterpret_cast<uint32_t *>(sf[dr] + cells);
  }
  const int first = mode == 1 ? ffh::kLevelInit : (mode == 2 ? ffh::kLevelSeed : ffh::kLevelContinue);
  return from_hip(run_level_blocked(k, W, H, level, params, first, (hipStream_t)stream, sf, sc));
}

ff_status ff_cost_f32_fwd(const float *f1, const float *f2, int32_t W, int32_t H, int32_t n, int32_t radius,
                          const int32_t *entries, int32_t count, float *cost, void *stream) {
  if (!f1 || !f2 || (count > 0 && (!entries || !cost)) || !dims_ok(W, H) || !is_pow2(n) || radius < 0 ||
      radius > 7 || count < 0)
    return FF_ERR_ARG;
  ffh::CostArgs a{};
  a.f1 = f1;
  a.f2 = f2;
  a.entries = reinterpret_cast<const int4 *>(entries);
  a.count = count;
  a.W = W;
  a.H = H;
  a.n = n;
  a.radius = radius;
  a.cost = cost;
  return from_hip(ffh::launch_cost_fwd(a, (hipStream_t)stream));
}

ff_status ff_cost_f32_bwd(const float *f1, const float *f2, int32_t W, int32_t H, int32_t n, int32_t radius,
                          const int32_t *entries, int32_t count, const float *grad_cost, int64_t *acc_scratch,
                          float *grad_f1, float *grad_f2, void *stream) {
  if (!f1 || !f2 || (count > 0 && (!entries || !grad_cost)) || !acc_scratch || !grad_f1 || !grad_f2 ||
      !dims_ok(W, H) || !is_pow2(n) || radius < 0 || radius > 7 || count < 0)
    return FF_ERR_ARG;
  ffh::CostArgs a{};
  a.f1 = f1;
  a.f2 = f2;
  a.entries = reinterpret_cast<const int4 *>(entries);
  a.count = count;
  a.W = W;
  a.H = H;
  a.n = n;
  a.radius = radius;
  a.grad_cost = grad_cost;
  a.acc1 = acc_scratch;
  a.acc2 = acc_scratch + (size_t)W * H * 16;
  a.overflow = acc_scratch + (size_t)2 * W * H * 16;
  a.grad_f1 = grad_f1;
  a.grad_f2 = grad_f2;
  return from_hip(ffh::launch_cost_bwd(a, (hipStream_t)stream));
}

// ---- batches -------------------------------------------------------------

static bool batch_ok(const ff_pair *pairs, int32_t npairs, const ff_params *p) {
  if (!pairs || npairs < 1 || npairs > ffh::kMaxBatch || !params_ok(p)) return false;
  for (int i = 0; i < npairs; ++i) {
    const ff_pair &q = pairs[i];
    if (!q.img1 || !q.img2 || !q.flow_fwd || !q.flow_bwd || !q.cost_fwd || !q.cost_bwd || !q.keep_fwd ||
        !nn_dims_ok(q.W, q.H))
      return false;
  }
  return true;
}

size_t ff_batch_workspace_bytes(const ff_pair *pairs, int32_t npairs, const ff_params *params) {
  if (!batch_ok(pairs, npairs, params)) return 0;
  size_t total = 0;
  for (int i = 0; i < npairs; ++i) total = align256(total + layout(pairs[i].W, pairs[i].H, params).total);
  return total;
}

size_t ff_batch_table_bytes(int32_t npairs) {
  return (npairs < 1 || npairs > ffh::kMaxBatch) ? 0 : sizeof(ffh::BatchPair) * (size_t)npairs;
}

ff_status ff_batch_table(const ff_pair *pairs, int32_t npairs, const ff_params *params, void *ws, size_t ws_bytes,
                         void *table_host, size_t table_bytes) {
  if (!batch_ok(pairs, npairs, params) || !ws || !table_host) return FF_ERR_ARG;
  if (ws_bytes < ff_batch_workspace_bytes(pairs, npairs, params) || table_bytes < ff_batch_table_bytes(npairs))
    return FF_ERR_WORKSPACE;
  ffh::BatchPair *tab = static_cast<ffh::BatchPair *>(table_host);
  char *base = static_cast<char *>(ws);
  size_t off = 0;
  const int L = params->levels;
  for (int i = 0; i < npairs; ++i) {
    const ff_pair &q = pairs[i];
    const Layout lay = layout(q.W, q.H, params);
    char *b = base + off;
    ffh::BatchPair t;
    std::memset(&t, 0, sizeof(t));
    t.img[0] = q.img1;
    t.img[1] = q.img2;
    t.W = q.W;
    t.H = q.H;
    for (int im = 0; im < 2; ++im) {
      for (int lv = 0; lv < L; ++lv) {
        const size_t z = (size_t)(im * L + lv);
        t.hsum[im][lv] = reinterpret_cast<uint16_t *>(b + lay.hsum) + z * lay.N;
        t.blur[im][lv] = reinterpret_cast<uint8_t *>(b + lay.blur) + z * lay.N;
        t.desc[im][lv] = reinterpret_cast<uint8_t *>(b + lay.desc[im][lv]);
        t.wform[im][lv] = reinterpret_cast<uint8_t *>(b + lay.wform[im][lv]);
      }
      t.desc1[im] = reinterpret_cast<uint8_t *>(b + lay.desc1) + (size_t)im * lay.N * 16;
      t.nb[im] = reinterpret_cast<int32_t *>(b + lay.nb) + (size_t)im * lay.Npad;
      t.keys[im] = reinterpret_cast<uint64_t *>(b + lay.keys) + (size_t)im * lay.M;
    }
    t.gflow[0][0] = reinterpret_cast<int32_t *>(q.flow_fwd);
    t.gflow[0][1] = reinterpret_cast<int32_t *>(q.flow_bwd);
    t.gcost[0][0] = q.cost_fwd;
    t.gcost[0][1] = q.cost_bwd;
    size_t g = lay.grids;
    for (int lv = 1; lv < L; ++lv) {
      const size_t cells = (size_t)ceil_div(q.W, 1 << lv) * ceil_div(q.H, 1 << lv);
      for (int dr = 0; dr < 2; ++dr) {
        t.gflow[lv][dr] = reinterpret_cast<int32_t *>(b + g) + (size_t)dr * 2 * cells;
        t.gcost[lv][dr] = reinterpret_cast<uint32_t *>(t.gflow[lv][dr] + cells);
      }
      g = align256(g + 2 * cells * 2 * sizeof(uint32_t));
    }
    carve_second_grids(b, lay.sgrids, q.W, q.H, L, t.sflow, t.scost);
    t.keep[0] = q.keep_fwd;
    t.keep[1] = q.keep_bwd;
    t.evals = reinterpret_cast<unsigned long long *>(q.n_evals ? q.n_evals
                                                               : reinterpret_cast<uint64_t *>(b + lay.evals));
    tab[i] = t;
    off = align256(off + lay.total);
  }
  return FF_OK;
}

ff_status ff_flow_fields_batched(const ff_pair *pairs, int32_t npairs, const ff_params *params, const void *table,
                                 void *ws, size_t ws_bytes, void *stream) {
  if (!batch_ok(pairs, npairs, params) || !table || !ws || !(params->eps >= 0.0f)) return FF_ERR_ARG;
  if (ws_bytes < ff_batch_workspace_bytes(pairs, npairs, params)) return FF_ERR_WORKSPACE;
  if (params->radius != 3 || params->subpixel || params->nn_l > 1 || params->raster || params->fast_x2 ||
      params->subscales)
    return FF_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  const int L = params->levels, nc = 1 << (L - 1);
  ffh::BatchStage st{};
  st.pairs = static_cast<const ffh::BatchPair *>(table);
  st.npairs = npairs;
  st.L = L;
  auto fill = [&](auto items_of) {
    st.prefix[0] = 0;
    for (int i = 0; i < npairs; ++i) st.prefix[i + 1] = st.prefix[i] + items_of(pairs[i].W, pairs[i].H);
    st.total = st.prefix[npairs];
  };
  hipError_t e;
  // descriptors: (pair, image * L + scale, row)
  fill([&](int, int H) { return 2 * L * H; });
  if ((e = ffh::launch_batch_descriptors(st, s)) != hipSuccess) return FF_ERR_LAUNCH;
  // NN: norms (pair, image, 256 refs), keys (pair, direction, 256 queries), NN items
  ffh::BatchStage norms = st, keysf = st, nn = st;
  norms.n = keysf.n = nn.n = nc;
  {
    auto set = [&](ffh::BatchStage &b, auto items_of) {
      b.prefix[0] = 0;
      for (int i = 0; i < npairs; ++i) b.prefix[i + 1] = b.prefix[i] + items_of(pairs[i].W, pairs[i].H);
      b.total = b.prefix[npairs];
    };
    set(norms, [&](int W, int H) { return 2 * (int)((((size_t)W * H + 31) / 32 * 32 + 255) / 256); });
    set(keysf, [&](int W, int H) { return 2 * ((ceil_div(W, nc) * ceil_div(H, nc) + 255) / 256); });
    set(nn, [&](int W, int H) { return ffh::batch_nn_items(W, H, L); });
  }
  if ((e = ffh::launch_batch_nn(norms, keysf, nn, s)) != hipSuccess) return FF_ERR_LAUNCH;
  // scales, coarse to fine: one persistent launch per run of passes
  const ffh::Tuning tun = tuning_of(params->tuning);
  for (int lv = L - 1; lv >= 0; --lv) {
    const int n = 1 << lv;
    bool maps_fit = true;
    for (int i = 0; i < npairs; ++i) maps_fit = maps_fit && ffh::level_map_fits(pairs[i].W, pairs[i].H, lv);
    // work items of the kernel that will run (a variant's fallback may tile differently)
    fill([&](int W, int H) {
      return 2 * ffh::level_tiles(ceil_div(W, n), ceil_div(H, n), tun.variant[lv], maps_fit);
    });
    st.n = n;
    st.lv = lv;
    ffh::LevelKArgs k{};
    k.ndir = 2;
    k.n = n;
    k.level = lv;
    const ScaleSteps sst = scale_steps(params, lv);
    k.Rn = sst.Rn;
    k.Rnp = sst.Rnp;
    k.P = sst.P;
    k.seed = params->seed;
    k.T = sst.total();
    k.variant = tun.variant[lv];
    int runs[64][2];
    const int m = level_runs(tun, lv, k.T, 0, runs);
    for (int r = 0; r < m; ++r) {
      // runs alternate between the two grid buffers; the last writes gflow/gcost
      st.dst = ((m - 1 - r) & 1) ? 1 : 0;
      st.src = st.dst ^ 1;
      ffh::level_halo(runs[r][0], runs[r][1], k.halo);
      k.t_begin = runs[r][0];
      k.t_end = runs[r][1];
      k.mode = r > 0 ? ffh::kLevelContinue : (lv == L - 1 ? ffh::kLevelInit : ffh::kLevelSeed);
      if ((e = ffh::launch_batch_level(k, st, maps_fit, s)) != hipSuccess) return FF_ERR_LAUNCH;
    }
  }
  fill([&](int, int H) { return 2 * H; });
  return from_hip(ffh::launch_batch_consistency(st, params->eps, s));
}

// ---- Flow Fields on learned float features ----------------------------------

struct LayoutF32 {
  size_t q, qscratch, nb, keys, grids, sgrids, evals, pf[2][kMaxLevels], total;
  size_t N, Npad, M;
};

static LayoutF32 layout_f32(int W, int H, const ff_params *p) {
  LayoutF32 l{};
  l.N = (size_t)W * H;
  l.Npad = (l.N + 31) & ~(size_t)31;
  const int nc = 1 << (p->levels - 1);
  l.M = (size_t)ceil_div(W, nc) * ceil_div(H, nc);
  size_t off = 0;
  l.q = off; off = align256(off + 2 * l.N * 16);
  l.qscratch = off; off = align256(off + ffh::quantize_scratch_bytes());
  l.nb = off; off = align256(off + 2 * l.Npad * sizeof(int32_t));
  l.keys = off; off = align256(off + 2 * l.M * sizeof(uint64_t));
  l.grids = off;
  for (int lv = 1; lv < p->levels; ++lv) {
    const size_t cells = (size_t)ceil_div(W, 1 << lv) * ceil_div(H, 1 << lv);
    off = align256(off + 2 * cells * 2 * sizeof(uint32_t));
  }
  l.sgrids = off;
  for (int lv = 0; lv < p->levels; ++lv) {
    const size_t cells = (size_t)ceil_div(W, 1 << lv) * ceil_div(H, 1 << lv);
    off = align256(off + 2 * cells * 2 * sizeof(uint32_t));
  }
  l.evals = off; off = align256(off + 2 * sizeof(uint64_t));
  if (p->radius == 3)  // padded float maps of the blocked level kernel
    for (int im = 0; im < 2; ++im)
      for (int lv = 0; lv < p->levels; ++lv) {
        l.pf[im][lv] = off;
        off = align256(off + desc_map_bytes(W, H, 1 << lv) * 4);
      }
  l.total = off;
  return l;
}

size_t ff_workspace_bytes_f32(int32_t W, int32_t H, const ff_params *params) {
  if (!nn_dims_ok(W, H) || !params_ok(params)) return 0;
  return layout_f32(W, H, params).total;
}

ff_status ff_flow_fields_f32(const float *const *feat1, const float *const *feat2, int32_t W, int32_t H,
                             const ff_params *params, void *ws, size_t ws_bytes, int16_t *flow_fwd, int16_t *flow_bwd,
                             uint32_t *cost_fwd, uint32_t *cost_bwd, uint8_t *keep_fwd, uint8_t *keep_bwd,
                             uint64_t *n_evals, void *stream) {
  if (!feat1 || !feat2 || !ws || !flow_fwd || !flow_bwd || !cost_fwd || !cost_bwd || !keep_fwd || !nn_dims_ok(W, H) ||
      !params_ok(params) || !(params->eps >= 0.0f))
    return FF_ERR_ARG;
  const int L = params->levels, r = params->radius;
  if (params->subpixel || params->nn_l > 1 || params->raster || params->fast_x2 || params->subscales)
    return FF_ERR_UNSUPPORTED;
  for (int lv = 0; lv < L; ++lv)
    if (!feat1[lv] || !feat2[lv]) return FF_ERR_ARG;
  const LayoutF32 lay = layout_f32(W, H, params);
  if (ws_bytes < lay.total) return FF_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char *base = static_cast<char *>(ws);
  hipError_t e;
  // bytes of the level-1 features for the matrix-core NN seed
  // (one range over both images: equal feature values become equal bytes)
  uint8_t *q[2];
  for (int im = 0; im < 2; ++im) q[im] = reinterpret_cast<uint8_t *>(base + lay.q) + (size_t)im * lay.N * 16;
  if ((e = ffh::launch_quantize_pair(feat1[0], feat2[0], (long long)lay.N * 16,
                                     reinterpret_cast<float *>(base + lay.qscratch), q[0], q[1], s)) != hipSuccess)
    return FF_ERR_LAUNCH;
  uint64_t *evals = n_evals ? n_evals : reinterpret_cast<uint64_t *>(base + lay.evals);
  if ((e = ffh::launch_fill_u64(evals, 0, 2, s)) != hipSuccess) return FF_ERR_LAUNCH;
  int32_t *gflow[kMaxLevels][2];
  uint32_t *gcost[kMaxLevels][2];
  gflow[0][0] = reinterpret_cast<int32_t *>(flow_fwd);
  gflow[0][1] = reinterpret_cast<int32_t *>(flow_bwd);
  gcost[0][0] = cost_fwd;
  gcost[0][1] = cost_bwd;
  size_t off = lay.grids;
  for (int lv = 1; lv < L; ++lv) {
    const size_t cells = (size_t)ceil_div(W, 1 << lv) * ceil_div(H, 1 << lv);
    for (int dr = 0; dr < 2; ++dr) {
      gflow[lv][dr] = reinterpret_cast<int32_t *>(base + off) + (size_t)dr * 2 * cells;
      gcost[lv][dr] = reinterpret_cast<uint32_t *>(gflow[lv][dr] + cells);
    }
    off = align256(off + 2 * cells * 2 * sizeof(uint32_t));
  }
  const int nc = 1 << (L - 1);
  uint64_t *keys = reinterpret_cast<uint64_t *>(base + lay.keys);
  int32_t *nb = reinterpret_cast<int32_t *>(base + lay.nb);
  ffh::NNArgs nn{};
  nn.ndir = 2;
  nn.W = W;
  nn.H = H;
  nn.nc = nc;
  nn.Wc = ceil_div(W, nc);
  nn.M = (int)lay.M;
  nn.N = (int)lay.N;
  for (int dr = 0; dr < 2; ++dr) nn.dir[dr] = {q[dr], q[dr ^ 1], nb + (size_t)dr * lay.Npad, keys + (size_t)dr * lay.M};
  if ((e = ffh::launch_nn(nn, s)) != hipSuccess) return FF_ERR_LAUNCH;
  const float *const *feat[2] = {feat1, feat2};
  if (r == 3) {
    // temporally blocked level kernels on padded, phase-ordered float maps
    const uint8_t *pf[2][kMaxLevels];
    for (int im = 0; im < 2; ++im)
      for (int lv = 0; lv < L; ++lv) {
        float *m = reinterpret_cast<float *>(base + lay.pf[im][lv]);
        if ((e = ffh::launch_pad_features(feat[im][lv], W, H, 1 << lv, m, s)) != hipSuccess) return FF_ERR_LAUNCH;
        pf[im][lv] = reinterpret_cast<const uint8_t *>(m);
      }
    int32_t *sflow[kMaxLevels][2];
    uint32_t *scost[kMaxLevels][2];
    carve_second_grids(base, lay.sgrids, W, H, L, sflow, scost);
    ffh::LevelKArgs k{};
    k.ndir = 2;
    k.fcost = 1;
    for (int dr = 0; dr < 2; ++dr) {
      k.dir[dr].n_evals = reinterpret_cast<unsigned long long *>(evals + dr);
      k.dir[dr].stream_id = dr;
    }
    for (int lv = L - 1; lv >= 0; --lv) {
      for (int dr = 0; dr < 2; ++dr) {
        k.dir[dr].Da = pf[dr][lv];
        k.dir[dr].Db = pf[dr ^ 1][lv];
        k.dir[dr].flow = gflow[lv][dr];
        k.dir[dr].cost = gcost[lv][dr];
        k.dir[dr].nn_key = keys + (size_t)dr * lay.M;
        k.dir[dr].cflow = lv + 1 < L ? gflow[lv + 1][dr] : nullptr;
        k.dir[dr].ccost = lv + 1 < L ? gcost[lv + 1][dr] : nullptr;
      }
      const int mode = lv == L - 1 ? ffh::kLevelInit : ffh::kLevelSeed;
      if ((e = run_level_blocked(k, W, H, lv, params, mode, s, sflow[lv], scost[lv])) != hipSuccess)
        return FF_ERR_LAUNCH;
    }
    return from_hip(ffh::launch_consistency(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, params->eps, keep_fwd,
                                            keep_bwd, s));
  }
  ffh::LevelArgs a{};
  a.ndir = 2;
  a.fcost = 1;
  a.W = W;
  a.H = H;
  a.radius = r;
  a.seed = params->seed;
  for (int dr = 0; dr < 2; ++dr) {
    a.dir[dr].n_evals = reinterpret_cast<unsigned long long *>(evals + dr);
    a.dir[dr].stream_id = dr;
  }
  for (int lv = L - 1; lv >= 0; --lv) {
    for (int dr = 0; dr < 2; ++dr) {
      a.dir[dr].Da = feat[dr][lv];
      a.dir[dr].Db = feat[dr ^ 1][lv];
      a.dir[dr].flow = gflow[lv][dr];
      a.dir[dr].cost = gcost[lv][dr];
      a.dir[dr].nn_key = keys + (size_t)dr * lay.M;
      a.dir[dr].Dq1 = q[dr];
      a.dir[dr].cflow = lv + 1 < L ? gflow[lv + 1][dr] : nullptr;
      a.dir[dr].ccost = lv + 1 < L ? gcost[lv + 1][dr] : nullptr;
    }
    if ((e = run_level_steps(a, W, H, lv, L, params, s)) != hipSuccess) return FF_ERR_LAUNCH;
  }
  return from_hip(ffh::launch_consistency(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, params->eps, keep_fwd,
                                          keep_bwd, s));
}

// ---- learned descriptor network ------------------------------------------

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

static bool conv_shape_ok(int B, int H, int W, int cin, int cout) {
  return B >= 1 && dims_ok(W, H) && (long long)B * H * W < (1ll << 31) &&
         ((cin == 1 && cout == 32) || (cin == 32 && cout == 32) || (cin == 32 && cout == 16) ||
          (cin == 16 && cout == 32));
}

ff_status ff_conv3x3_fwd(const uint16_t *in, int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout,
                         const uint16_t *w, const float *bias, int32_t relu, float *out_f32, uint16_t *out_bf16,
                         void *stream) {
  if (!in || !w || (!out_f32 && !out_bf16) || !conv_shape_ok(B, H, W, cin, cout)) return FF_ERR_ARG;
  if (cin >= 16 && !aligned16(in)) return FF_ERR_ARG;  // 16-byte loads of input channel chunks
  ffh::ConvArgs a{};
  a.in = in;
  a.w = w;
  a.bias = bias;
  a.B = B;
  a.H = H;
  a.W = W;
  a.cin = cin;
  a.cout = cout;
  a.relu = relu != 0;
  a.out_f32 = out_f32;
  a.out_bf16 = out_bf16;
  return from_hip(ffh::launch_conv_fwd(a, (hipStream_t)stream));
}

ff_status ff_conv3x3_bwd_data(const uint16_t *gout, int32_t B, int32_t H, int32_t W, int32_t cin, int32_t cout,
                              const uint16_t *w, uint16_t *wflip_scratch, float *gin_f32, uint16_t *gin_bf16,
                              void *stream) {
  if (!gout || !w || !wflip_scratch || (!gin_f32 && !gin_bf16) || !conv_shape_ok(B, H, W, cout, cin))
    return FF_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  if (ffh::launch_weight_flip(w, wflip_scratch, cin, cout, s) != hipSuccess) return FF_ERR_LAUNCH;
  return ff_conv3x3_fwd(gout, B, H, W, cout, cin, wflip_scratch, nullptr, 0, gin_f32, gin_bf16, stream);
}

size_t ff_conv3x3_wgrad_scratch_bytes(int32_t B, int32_t H, int32_t cin, int32_t cout) {
  if (B < 1 || H < 1) return 0;
  return (size_t)ffh::wgrad_blocks(B, H) * (size_t)(cout * 9 * cin + cout) * sizeof(float);
}

ff_status ff_conv3x3_bwd_weight(const uint16_t *in, const float *gout, int32_t B, int32_t H, int32_t W, int32_t cin,
                                int32_t cout, float *scratch, size_t scratch_bytes, float *gw, float *gbias,
                                void *stream) {
  if (!in || !gout || !scratch || !gw || !conv_shape_ok(B, H, W, cin, cout) || cin == 16) return FF_ERR_ARG;
  // 16-byte loads: 8 input channels, 4 gradients at a time
  if ((cin > 1 && !aligned16(in)) || !aligned16(gout)) return FF_ERR_ARG;
  if (scratch_bytes < ff_conv3x3_wgrad_scratch_bytes(B, H, cin, cout)) return FF_ERR_WORKSPACE;
  ffh::ConvArgs a{};
  a.in = in;
  a.gout = gout;
  a.B = B;
  a.H = H;
  a.W = W;
  a.cin = cin;
  a.cout = cout;
  a.partial = scratch;
  return from_hip(ffh::launch_wgrad(a, gw, gbias, (hipStream_t)stream));
}

ff_status ff_relu_bwd(const uint16_t *act, const float *grad, int64_t count, float *grad_out, uint16_t *grad_out_bf16,
                      void *stream) {
  if (!grad || (!grad_out && !grad_out_bf16) || count < 0) return FF_ERR_ARG;
  return from_hip(ffh::launch_relu_bwd(act, grad, grad_out, grad_out_bf16, count, (hipStream_t)stream));
}

ff_status ff_f32_to_bf16(const float *x, int64_t count, uint16_t *y, void *stream) {
  if (!x || !y || count < 0) return FF_ERR_ARG;
  return from_hip(ffh::launch_f32_to_bf16(x, y, count, (hipStream_t)stream));
}

ff_status ff_image_to_bf16(const uint8_t *img, int64_t count, uint16_t *out, void *stream) {
  if (!img || !out || count < 0) return FF_ERR_ARG;
  return from_hip(ffh::launch_image_to_bf16(img, out, count, (hipStream_t)stream));
}

ff_status ff_adam_step(float *param, const float *grad, float *m, float *v, int32_t count, float lr, float beta1,
                       float beta2, float eps, int32_t step, uint16_t *param_bf16, void *stream) {
  if (!param || !grad || !m || !v || count < 0 || step < 1 || !(lr >= 0.0f)) return FF_ERR_ARG;
  return from_hip(ffh::launch_adam(param, grad, m, v, count, lr, beta1, beta2, eps, step, param_bf16,
                                   (hipStream_t)stream));
}

ff_status ff_descnet_fwd(const uint16_t *in, int32_t B, int32_t H, int32_t W, const uint16_t *w1, const float *b1,
                         const uint16_t *w2, const float *b2, const uint16_t *w3, const float *b3, int32_t normalize,
                         float delta, float *out, void *stream) {
  if (!in || !w1 || !b1 || !w2 || !b2 || !w3 || !b3 || !out || B < 1 || !dims_ok(W, H) ||
      (long long)B * H * W >= (1ll << 31) || (normalize && !(delta > 0.0f)) || !aligned16(w2) || !aligned16(w3) ||
      !aligned16(out))
    return FF_ERR_ARG;
  ffh::NetArgs a{};
  a.in = in;
  a.w1 = w1;
  a.w2 = w2;
  a.w3 = w3;
  a.b1 = b1;
  a.b2 = b2;
  a.b3 = b3;
  a.B = B;
  a.H = H;
  a.W = W;
  a.normalize = normalize != 0;
  a.delta = delta;
  a.out = out;
  return from_hip(ffh::launch_descnet_fwd(a, (hipStream_t)stream));
}

ff_status ff_l2norm16_fwd(const float *feat, int64_t pixels, float delta, float *out, float *inv_norm, void *stream) {
  if (!feat || !out || pixels < 0 || !(delta > 0.0f) || !aligned16(feat) || !aligned16(out)) return FF_ERR_ARG;
  return from_hip(ffh::launch_l2norm16_fwd(feat, pixels, delta, out, inv_norm, (hipStream_t)stream));
}

ff_status ff_l2norm16_bwd(const float *out, const float *inv_norm, const float *grad, int64_t pixels, float *grad_in,
                          void *stream) {
  if (!out || !inv_norm || !grad || !grad_in || pixels < 0 || !aligned16(out) || !aligned16(grad) ||
      !aligned16(grad_in))
    return FF_ERR_ARG;
  return from_hip(ffh::launch_l2norm16_bwd(out, inv_norm, grad, pixels, grad_in, (hipStream_t)stream));
}

ff_status ff_triplet_hinge(const float *cost, int32_t m, float margin, float scale, float weight, float *grad_cost,
                           float *loss, void *stream) {
  if (!cost || !grad_cost || !loss || m < 0) return FF_ERR_ARG;
  return from_hip(ffh::launch_triplet_hinge(cost, m, margin, scale, weight, grad_cost, loss, (hipStream_t)stream));
}

size_t ff_quantize_scratch_bytes(void) { return ffh::quantize_scratch_bytes(); }

ff_status ff_quantize_u8(const float *f, int64_t count, float *scratch, uint8_t *q, void *stream) {
  if (!f || !scratch || !q || count < 0) return FF_ERR_ARG;
  return from_hip(ffh::launch_quantize(f, count, scratch, q, (hipStream_t)stream));
}

ff_status ff_quantize_pair_u8(const float *f1, const float *f2, int64_t count, float *scratch, uint8_t *q1,
                              uint8_t *q2, void *stream) {
  if (!f1 || !f2 || !scratch || !q1 || !q2 || count < 0) return FF_ERR_ARG;
  return from_hip(ffh::launch_quantize_pair(f1, f2, count, scratch, q1, q2, (hipStream_t)stream));
}

int32_t ff_level_variant_count(void) { return ffh::level_variant_count(); }

int32_t ff_level_variant_count_f32(void) { return ffh::level_variant_count_f32(); }

void ff_default_tuning(ff_tuning *out) {
  if (!out) return;
  const ffh::Tuning &t = ffh::default_tuning();
  for (int k = 0; k < ffh::kTuneScales; ++k) {
    out->variant[k] = t.variant[k];
    out->passes[k] = t.passes[k];
    out->variant_f32[k] = t.variant_f32[k];
    out->passes_f32[k] = t.passes_f32[k];
  }
}

int32_t ff_level_launches(const ff_tuning *tuning, int32_t iters, int32_t log2n, int32_t cost_kind) {
  const ffh::Tuning tun = tuning_of(tuning);
  if (iters < 1 || iters > 64 || log2n < 0 || log2n >= ffh::kTuneScales || (cost_kind != 0 && cost_kind != 1) ||
      !ffh::tuning_ok(tun))
    return -1;
  int runs[64][2];
  return level_runs(tun, log2n, iters, cost_kind, runs);
}

size_t ff_workspace_bytes(int32_t W, int32_t H, const ff_params *params) {
  if (!nn_dims_ok(W, H) || !params_ok(params)) return 0;
  return layout(W, H, params).total;
}

ff_status ff_flow_fields(const uint8_t *img1, const uint8_t *img2, int32_t W, int32_t H, const ff_params *params,
                         void *ws, size_t ws_bytes, int16_t *flow_fwd, int16_t *flow_bwd, uint32_t *cost_fwd,
                         uint32_t *cost_bwd, uint8_t *keep_fwd, uint8_t *keep_bwd, uint64_t *n_evals, void *stream) {
  // forward field only: every backward output and both masks NULL
  const bool fwd_only = !flow_bwd && !cost_bwd && !keep_fwd && !keep_bwd;
  if (!img1 || !img2 || !ws || !flow_fwd || !cost_fwd || (!fwd_only && (!flow_bwd || !cost_bwd || !keep_fwd)) ||
      !nn_dims_ok(W, H) || !params_ok(params) || !(params->eps >= 0.0f) || !sub_dims_ok(params, W, H))
    return FF_ERR_ARG;
  const int sb = params->subpixel;  // flows in 1/2^sb px
  const int nd = fwd_only ? 1 : 2;  // directions computed
  const Layout lay = layout(W, H, params);
  if (ws_bytes < lay.total) return FF_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  const int L = params->levels, r = params->radius;
  const int lmin = params->fast_x2 ? 1 : 0;  // finest scale run (Fast x2: scale 2)
  char *base = static_cast<char *>(ws);
  const uint8_t *img[2] = {img1, img2};

  // descriptors of both images at every scale; the weight-class row maps
  // only where the table's level-kernel variant evaluates on them
  const ffh::Tuning tun = tuning_of(params->tuning);
  auto wform_used = [&](int lv) {
    return lv >= lmin && params->subpixel == 0 && !params->raster && r == 3 && ffh::level_uses_wform(tun.variant[lv]);
  };
  uint8_t *desc[2][kMaxLevels], *desc1[2];
  ffh::DescJobs jobs{};
  jobs.W = W;
  jobs.H = H;
  jobs.count = 2 * L;
  for (int im = 0; im < 2; ++im) {
    desc1[im] = reinterpret_cast<uint8_t *>(base + lay.desc1) + (size_t)im * lay.N * 16;
    for (int lv = 0; lv < L; ++lv) {
      const int z = im * L + lv;
      desc[im][lv] = reinterpret_cast<uint8_t *>(base + lay.desc[im][lv]);
      // scales below lmin only give the NN its level-1 descriptors
      jobs.job[z] = {img[im], reinterpret_cast<uint16_t *>(base + lay.hsum) + (size_t)z * lay.N,
                     reinterpret_cast<uint8_t *>(base + lay.blur) + (size_t)z * lay.N,
                     lv < lmin ? nullptr : desc[im][lv], lv == 0 ? desc1[im] : nullptr,
                     wform_used(lv) ? reinterpret_cast<uint8_t *>(base + lay.wform[im][lv]) : nullptr, 1 << lv};
    }
  }
  hipError_t e = ffh::launch_descriptors(jobs, s);
  if (e != hipSuccess) return FF_ERR_LAUNCH;
  // sub-scales: the maps of patch scale 3n/2 (after the jobs above on the
  // same stream, so their row-sum and blur scratch can be reused)
  uint8_t *sdesc[2][kMaxLevels] = {};
  if (params->subscales && L > 2) {
    ffh::DescJobs sj{};
    sj.W = W;
    sj.H = H;
    for (int im = 0; im < 2; ++im)
      for (int lv = 1; lv + 1 < L; ++lv) {
        const int z = sj.count++;
        sdesc[im][lv] = reinterpret_cast<uint8_t *>(base + lay.sdesc[im][lv]);
        sj.job[z] = {img[im], reinterpret_cast<uint16_t *>(base + lay.hsum) + (size_t)z * lay.N,
                     reinterpret_cast<uint8_t *>(base + lay.blur) + (size_t)z * lay.N, sdesc[im][lv], nullptr, nullptr,
                     subscale_of(lv)};
      }
    if ((e = ffh::launch_descriptors(sj, s)) != hipSuccess) return FF_ERR_LAUNCH;
  }

  uint64_t *evals = n_evals ? n_evals : reinterpret_cast<uint64_t *>(base + lay.evals);
  if ((e = ffh::launch_fill_u64(evals, 0, 2, s)) != hipSuccess) return FF_ERR_LAUNCH;

  // level grids: the finest scale run lives in the caller's outputs
  int32_t *gflow[kMaxLevels][2];
  uint32_t *gcost[kMaxLevels][2];
  size_t off = lay.grids;
  for (int lv = 1; lv < L; ++lv) {
    const size_t cells = (size_t)ceil_div(W, 1 << lv) * ceil_div(H, 1 << lv);
    for (int dr = 0; dr < 2; ++dr) {
      gflow[lv][dr] = reinterpret_cast<int32_t *>(base + off) + (size_t)dr * 2 * cells;
      gcost[lv][dr] = reinterpret_cast<uint32_t *>(gflow[lv][dr] + cells);
    }
    off = align256(off + 2 * cells * 2 * sizeof(uint32_t));
  }
  gflow[lmin][0] = reinterpret_cast<int32_t *>(flow_fwd);
  gflow[lmin][1] = reinterpret_cast<int32_t *>(flow_bwd);
  gcost[lmin][0] = cost_fwd;
  gcost[lmin][1] = cost_bwd;

  // exact NN seeds of the coarsest grid, both directions
  const int nc = 1 << (L - 1);
  uint64_t *keys = reinterpret_cast<uint64_t *>(base + lay.keys);
  int32_t *nb = reinterpret_cast<int32_t *>(base + lay.nb);
  ffh::NNArgs nn{};
  nn.ndir = nd;
  nn.W = W;
  nn.H = H;
  nn.nc = nc;
  nn.Wc = ceil_div(W, nc);
  nn.M = (int)lay.M;
  nn.N = (int)lay.N;
  // references: every pixel, or (Fast x2) the pixels with even x and y
  const uint8_t *refs[2] = {desc1[0], desc1[1]};
  if (params->fast_x2) {
    nn.N = ceil_div(W, 2) * ceil_div(H, 2);
    for (int im = 0; im < 2; ++im) {
      uint8_t *ev = reinterpret_cast<uint8_t *>(base + lay.desc1e) + (size_t)im * nn.N * 16;
      if ((e = ffh::launch_gather_even(desc1[im], ev, W, H, s)) != hipSuccess) return FF_ERR_LAUNCH;
      refs[im] = ev;
    }
  }
  for (int dr = 0; dr < nd; ++dr)
    nn.dir[dr] = {desc1[dr], refs[dr ^ 1], nb + (size_t)dr * lay.Npad, keys + (size_t)dr * lay.M};
  if ((e = ffh::launch_nn(nn, s)) != hipSuccess) return FF_ERR_LAUNCH;
  if (params->fast_x2 && params->nn_l <= 1)
    for (int dr = 0; dr < nd; ++dr)
      if ((e = ffh::launch_remap_even(keys + (size_t)dr * lay.M, nn.M, W, s)) != hipSuccess) return FF_ERR_LAUNCH;
  if (params->nn_l > 1) {
    // seed rerank among the nn_l nearest pixels (Eq. 1, Eq. 4)
    ffh::TopLArgs tl{};
    tl.ndir = nd;
    tl.l = params->nn_l;
    tl.W = W;
    tl.H = H;
    tl.nc = nc;
    tl.Wc = nn.Wc;
    tl.M = nn.M;
    tl.N = nn.N;
    tl.even_refs = params->fast_x2;
    const uint64_t *cand[2];
    for (int dr = 0; dr < nd; ++dr) {
      ffh::TopLDir &d = tl.dir[dr];
      d.Dq = desc1[dr];
      d.Dr = refs[dr ^ 1];
      d.nb = nb + (size_t)dr * lay.Npad;
      d.nn_key = keys + (size_t)dr * lay.M;
      d.keys = reinterpret_cast<uint64_t *>(base + lay.topl + (size_t)dr * ffh::topl_scratch_bytes((int)lay.M));
      d.cand = reinterpret_cast<uint64_t *>(base + lay.cand) + (size_t)dr * lay.M * params->nn_l;
      cand[dr] = d.cand;
    }
    if ((e = ffh::launch_topl(tl, s)) != hipSuccess) return FF_ERR_LAUNCH;
    ffh::LevelArgs ra{};
    ra.ndir = nd;
    ra.fcost = sb ? 2 : 0;
    ra.W = W;
    ra.H = H;
    ra.n = nc;
    ra.Wn = ceil_div(W, nc);
    ra.Hn = ceil_div(H, nc);
    ra.radius = r;
    for (int dr = 0; dr < nd; ++dr) {
      ra.dir[dr].Da = desc[dr][L - 1];
      ra.dir[dr].Db = desc[dr ^ 1][L - 1];
      ra.dir[dr].Dq1 = desc1[dr];
      ra.dir[dr].nn_key = keys + (size_t)dr * lay.M;
      ra.dir[dr].n_evals = reinterpret_cast<unsigned long long *>(evals + dr);
    }
    if ((e = ffh::launch_rerank(ra, cand, params->nn_l, s)) != hipSuccess) return FF_ERR_LAUNCH;
  }

  // stages coarse to fine: (scale 2^lv, patch scale m, entry), entry 0:
  // the NN initialisation, 1: the same grid at a new patch scale, 2: the
  // hand-over from the coarser grid
  int stage_lv[2 * kMaxLevels], stage_m[2 * kMaxLevels], stage_entry[2 * kMaxLevels], nst = 0;
  if (params->subscales) {
    nst = subscale_stages(L, stage_lv, stage_m);
  } else {
    for (int lv = L - 1; lv >= lmin; --lv, ++nst) {
      stage_lv[nst] = lv;
      stage_m[nst] = 1 << lv;
    }
  }
  for (int k = 0; k < nst; ++k) stage_entry[k] = k == 0 ? 0 : (stage_lv[k - 1] == stage_lv[k] ? 1 : 2);

  if (sb == 0 && !params->raster && ffh::level_blocked_ok(W, H, L, r)) {
    // temporally blocked level kernels: one launch per run of passes (the
    // sub-scale stages, whose patch scale differs from the grid scale, one
    // launch per step)
    int32_t *sflow[kMaxLevels][2];
    uint32_t *scost[kMaxLevels][2];
    carve_second_grids(base, lay.sgrids, W, H, L, sflow, scost);
    ffh::LevelKArgs k{};
    k.ndir = nd;
    for (int dr = 0; dr < nd; ++dr) {
      k.dir[dr].n_evals = reinterpret_cast<unsigned long long *>(evals + dr);
      k.dir[dr].stream_id = dr;
    }
    for (int st = 0; st < nst; ++st) {
      const int lv = stage_lv[st], m = stage_m[st], entry = stage_entry[st];
      for (int dr = 0; dr < nd; ++dr) {
        k.dir[dr].Da = desc[dr][lv];
        k.dir[dr].Db = desc[dr ^ 1][lv];
        k.dir[dr].Wa = wform_used(lv) ? reinterpret_cast<const uint8_t *>(base + lay.wform[dr][lv]) : nullptr;
        k.dir[dr].Wb = wform_used(lv) ? reinterpret_cast<const uint8_t *>(base + lay.wform[dr ^ 1][lv]) : nullptr;
        k.dir[dr].flow = gflow[lv][dr];
        k.dir[dr].cost = gcost[lv][dr];
        k.dir[dr].nn_key = keys + (size_t)dr * lay.M;
        k.dir[dr].cflow = lv + 1 < L ? gflow[lv + 1][dr] : nullptr;
        k.dir[dr].ccost = lv + 1 < L ? gcost[lv + 1][dr] : nullptr;
      }
      const bool sub = m != (1 << lv);
      const bool stepwise = ffh::level_stepwise(tuning_of(params->tuning).variant[lv]);
      // a sub-scale stage on the blocked quad kernels: radius 3, its map
      // addressed with 32-bit offsets, not the last stage (the Fast step
      // count applies there), entered from the coarser grid
      if (sub && !stepwise && r == 3 && entry == 2 && st != nst - 1 &&
          (size_t)(W + 2 * ffk::desc_pad(m)) * (H + 2 * ffk::desc_pad(m)) * 16 < ((size_t)1 << 31)) {
        for (int dr = 0; dr < nd; ++dr) {
          k.dir[dr].Da = sdesc[dr][lv];
          k.dir[dr].Db = sdesc[dr ^ 1][lv];
          k.dir[dr].Wa = nullptr;
          k.dir[dr].Wb = nullptr;
        }
        if ((e = run_level_blocked(k, W, H, lv, params, ffh::kLevelSeed, s, sflow[lv], scost[lv], m)) != hipSuccess)
          return FF_ERR_LAUNCH;
        continue;
      }
      if (sub || stepwise || entry == 1) {
        ffh::LevelArgs a{};
        a.ndir = nd;
        for (int dr = 0; dr < nd; ++dr) {
          const ffh::LevelKDir &kd = k.dir[dr];
          a.dir[dr] = {sub ? sdesc[dr][lv] : kd.Da, sub ? sdesc[dr ^ 1][lv] : kd.Db, kd.flow, kd.cost, kd.cflow,
                       kd.ccost, kd.nn_key, desc1[dr], kd.n_evals, nullptr, dr};
        }
        if (sub || stepwise) {
          if ((e = run_stage(a, W, H, lv, m, entry, st == nst - 1, params, s)) != hipSuccess) return FF_ERR_LAUNCH;
          continue;
        }
        // the grid at its own patch scale again: costs re-evaluated, then
        // the blocked launches continue from that state
        a.W = W;
        a.H = H;
        a.n = a.ns = m;
        a.Wn = ceil_div(W, m);
        a.Hn = ceil_div(H, m);
        a.radius = r;
        if ((e = ffh::launch_rescore(a, s)) != hipSuccess) return FF_ERR_LAUNCH;
      }
      const int mode = entry == 0 ? ffh::kLevelInit : entry == 2 ? ffh::kLevelSeed : ffh::kLevelContinue;
      if ((e = run_level_blocked(k, W, H, lv, params, mode, s, sflow[lv], scost[lv])) != hipSuccess)
        return FF_ERR_LAUNCH;
    }
    if (fwd_only) return FF_OK;
    if (params->fast_x2)
      return from_hip(ffh::launch_consistency_grid(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, 2, params->eps,
                                                   keep_fwd, keep_bwd, s));
    return from_hip(ffh::launch_consistency(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, params->eps, keep_fwd,
                                            keep_bwd, s));
  }

  ffh::LevelArgs a{};
  a.ndir = nd;
  a.fcost = sb ? 2 : 0;
  a.W = W;
  a.H = H;
  a.radius = r;
  a.seed = params->seed;
  for (int dr = 0; dr < nd; ++dr) {
    a.dir[dr].n_evals = reinterpret_cast<unsigned long long *>(evals + dr);
    a.dir[dr].stream_id = dr;
  }
  if (params->subscales) {
    // stages (n, 3n/2), (n, n) for every scale below the coarsest but the finest
    for (int k = 0; k < nst; ++k) {
      const int lv = stage_lv[k], m = stage_m[k];
      for (int dr = 0; dr < nd; ++dr) {
        a.dir[dr].Da = m == (1 << lv) ? desc[dr][lv] : sdesc[dr][lv];
        a.dir[dr].Db = m == (1 << lv) ? desc[dr ^ 1][lv] : sdesc[dr ^ 1][lv];
        a.dir[dr].flow = gflow[lv][dr];
        a.dir[dr].cost = gcost[lv][dr];
        a.dir[dr].nn_key = keys + (size_t)dr * lay.M;
        a.dir[dr].Dq1 = desc1[dr];
        a.dir[dr].cflow = lv + 1 < L ? gflow[lv + 1][dr] : nullptr;
        a.dir[dr].ccost = lv + 1 < L ? gcost[lv + 1][dr] : nullptr;
      }
      if ((e = run_stage(a, W, H, lv, m, stage_entry[k], k == nst - 1, params, s)) != hipSuccess)
        return FF_ERR_LAUNCH;
    }
  } else {
    for (int lv = L - 1; lv >= lmin; --lv) {
      for (int dr = 0; dr < nd; ++dr) {
        a.dir[dr].Da = desc[dr][lv];
        a.dir[dr].Db = desc[dr ^ 1][lv];
        a.dir[dr].flow = gflow[lv][dr];
        a.dir[dr].cost = gcost[lv][dr];
        a.dir[dr].nn_key = keys + (size_t)dr * lay.M;
        a.dir[dr].Dq1 = desc1[dr];
        a.dir[dr].cflow = lv + 1 < L ? gflow[lv + 1][dr] : nullptr;
        a.dir[dr].ccost = lv + 1 < L ? gcost[lv + 1][dr] : nullptr;
      }
      if ((e = run_level_steps(a, W, H, lv, L, params, s)) != hipSuccess) return FF_ERR_LAUNCH;
    }
  }
  if (fwd_only) return FF_OK;
  if (params->fast_x2)
    return from_hip(ffh::launch_consistency_grid(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, 2, params->eps,
                                                 keep_fwd, keep_bwd, s));
  return from_hip(ffh::launch_consistency(flow_fwd, cost_fwd, flow_bwd, cost_bwd, W, H, params->eps, keep_fwd,
                                          keep_bwd, s, sb));
}

}  // extern "C"
