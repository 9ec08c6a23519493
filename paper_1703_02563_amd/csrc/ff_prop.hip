// Level-grid kernels of the Flow Fields schedule (Sec. 3.1, 3.2, 3.7).
//
//  * k_init_coarse: initial flow F = q - p of the coarsest grid from the NN
//    keys, cost E_nc (Eq. 1 / Eq. 4 with one candidate).
//  * k_seed_level:  coarse-to-fine hand-over: cells with even (i, j) are the
//    coarse cell's pixel and keep its flow (cost re-evaluated at scale n);
//    the rest start UNSET (Sec. 3.2).
//  * k_prop_half:   one checkerboard half-sweep of a propagation step
//    (Eq. 2): cells of one colour read only cells of the other colour, so
//    every cell of the colour updates in parallel.  Candidate order own,
//    horizontal source, vertical source; strictly lower cost wins.
//  * k_random_search: one random-search step (Sec. 3.1) with integer
//    offsets from the counter-based generator.
//  * k_consistency: forward-backward check (Sec. 3.7); k_consistency2 the
//    same against two backward fields; k_sparsify: one sample per q x q
//    region (Sec. 3.8).
//
// One lane per cell; both directions of a pair run in one launch
// (blockIdx.z).  Each kernel counts the patch-cost evaluations it performs
// with one atomic per wave.
#include <algorithm>

#include "ff_device.h"
#include "ff_internal.h"

namespace {

using ffk::clampi;
using ffk::kUnset;

template <int R, class Cost>
__global__ __launch_bounds__(256) void k_init_coarse(ffh::LevelArgs a) {
  const ffh::LevelDir d = a.dir[blockIdx.z];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int cells = a.Wn * a.Hn;
  int cnt = 0;
  if (m < cells) {
    const int i = m % a.Wn, j = m / a.Wn;
    const int x = i * a.n, y = j * a.n;
    const uint64_t key = d.nn_key[m];
    const uint32_t q = (uint32_t)key;
    const int dd = (int)(uint32_t)(key >> 32) - (1 << 20);
    const uint4 qa = reinterpret_cast<const uint4 *>(d.Dq1)[(size_t)y * a.W + x];
    const uint32_t w[4] = {qa.x, qa.y, qa.z, qa.w};
    int na = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int e = (int)((w[k] >> (8 * b)) & 0xFF) - 128;
        na += e * e;
      }
    const_cast<uint64_t *>(d.nn_key)[m] = ((uint64_t)(uint32_t)(dd + na) << 32) | q;
    // the seed is an integer flow, stored in the cost's flow unit
    const int fx = ((int)(q % (uint32_t)a.W) - x) * (1 << Cost::kSub), fy = ((int)(q / (uint32_t)a.W) - y) * (1 << Cost::kSub);
    d.flow[m] = ffk::pack_flow(fx, fy);
    d.cost[m] = Cost::template eval<R>(d.Da, d.Db,
                                   a.W, a.H, a.ns > 0 ? a.ns : a.n, x, y, fx, fy);
    cnt = 1;
  }
  ffk::wave_count_add(d.n_evals, cnt);
  ffk::wave_count_add2(d.n_work, cnt);
}

template <int R, class Cost>
__global__ __launch_bounds__(256) void k_seed_level(ffh::LevelArgs a) {
  const ffh::LevelDir d = a.dir[blockIdx.z];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (m < a.Wn * a.Hn) {
    const int i = m % a.Wn, j = m / a.Wn;
    int32_t f = 0;
    uint32_t c = kUnset;
    if (!((i | j) & 1)) {
      const int Wc = (a.Wn + 1) >> 1;
      const int kc = (j >> 1) * Wc + (i >> 1);
      if (d.ccost[kc] != kUnset) {
        f = d.cflow[kc];
        c = Cost::template eval<R>(d.Da, d.Db,
                               a.W, a.H, a.ns > 0 ? a.ns : a.n, i * a.n, j * a.n, ffk::flow_x(f), ffk::flow_y(f));
        cnt = 1;
      }
    }
    d.flow[m] = f;
    d.cost[m] = c;
  }
  ffk::wave_count_add(d.n_evals, cnt);
  ffk::wave_count_add2(d.n_work, cnt);
}

// Half-sweep of colour `colour` ((i + j) & 1 == colour) of propagation step
// `a.pass`.  Grid: x over half-columns, y over rows, z over directions.
template <int R, class Cost>
__global__ __launch_bounds__(256) void k_prop_half(ffh::LevelArgs a, int colour) {
  const ffh::LevelDir d = a.dir[blockIdx.z];
  const int kx = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int i = 2 * kx + ((colour + j) & 1);
  const int Wn = a.Wn, Hn = a.Hn, W = a.W, H = a.H, n = a.n, ns = a.ns > 0 ? a.ns : a.n;
  int cnt = 0, work = 0;
  if (i < Wn && j < Hn) {
    const int dir = a.pass & 3;
    const int hdi = (dir == 0 || dir == 3) ? -1 : 1;
    const int vdj = (dir == 0 || dir == 2) ? -1 : 1;
    const int k = j * Wn + i;
    const int x = i * n, y = j * n;
    const uint32_t c0 = d.cost[k];
    const int32_t f0 = d.flow[k];
    const bool set0 = c0 != kUnset;
    // horizontal source
    const int hi = i + hdi;
    bool hv = false;
    int32_t fh = 0;
    if (hi >= 0 && hi < Wn) {
      const int ks = j * Wn + hi;
      if (d.cost[ks] != kUnset) {
        fh = d.flow[ks];
        hv = !(set0 && fh == f0) && ffk::target_in<Cost::kSub>(W, H, x, y, ffk::flow_x(fh), ffk::flow_y(fh));
      }
    }
    // vertical source: validity except the "held flow" rule, which depends
    // on the horizontal outcome
    const int vj = j + vdj;
    bool vb = false;
    int32_t fv = 0;
    if (vj >= 0 && vj < Hn) {
      const int ks = vj * Wn + i;
      if (d.cost[ks] != kUnset) {
        fv = d.flow[ks];
        vb = ffk::target_in<Cost::kSub>(W, H, x, y, ffk::flow_x(fv), ffk::flow_y(fv));
      }
    }
    // E(p, fv) need not be computed in the shared pass when fv equals fh
    // (same evaluation) or the held flow f0 (then it is only evaluated if
    // the horizontal source replaced f0, which is rare)
    const bool vcomp = vb && !(hv && fv == fh) && !(set0 && fv == f0);
    uint32_t eh = 0, ev = 0;
    work = (int)hv + (int)vcomp;
    if (hv || vcomp)
      Cost::template eval2<R>(d.Da, d.Db, W, H, ns,
                          x, y, ffk::flow_x(fh), ffk::flow_y(fh), hv, ffk::flow_x(fv), ffk::flow_y(fv), vcomp,
                          eh, ev);
    uint32_t bc = c0;
    int32_t bf = f0;
    if (hv) {
      cnt = 1;
      if (eh < bc) { bc = eh; bf = fh; }
    }
    if (vb && (bc == kUnset || fv != bf)) {
      cnt += 1;
      uint32_t e;
      if (hv && fv == fh)
        e = eh;
      else if (vcomp)
        e = ev;
      else {  // fv == f0 after the horizontal source replaced it; the stored
              // cost of a caller-made state need not equal E(p, f0)
        e = Cost::template eval<R>(d.Da, d.Db, W, H,
                               ns, x, y, ffk::flow_x(fv), ffk::flow_y(fv));
        work += 1;
      }
      if (e < bc) { bc = e; bf = fv; }
    }
    if (bc != c0 || bf != f0) {
      d.cost[k] = bc;
      d.flow[k] = bf;
    }
  }
  ffk::wave_count_add(d.n_evals, cnt);
  ffk::wave_count_add2(d.n_work, work);
}

template <int R, class Cost>
__global__ __launch_bounds__(256) void k_random_search(ffh::LevelArgs a) {
  const ffh::LevelDir d = a.dir[blockIdx.z];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  int cnt = 0;
  if (i < a.Wn && j < a.Hn) {
    const int k = j * a.Wn + i;
    const uint32_t c0 = d.cost[k];
    if (c0 != kUnset) {
      int ox, oy;
      // offsets uniform on [-Rn, Rn]^2 in the cost's flow unit
      ffk::rs_offset(a.seed, d.stream_id, a.level, a.pass, j, i, a.Rn * (1 << Cost::kSub), ox, oy);
      const int32_t f0 = d.flow[k];
      const int fx = ffk::flow_x(f0) + ox, fy = ffk::flow_y(f0) + oy;
      const int x = i * a.n, y = j * a.n;
      if ((ox | oy) != 0 && ffk::target_in<Cost::kSub>(a.W, a.H, x, y, fx, fy)) {
        const uint32_t e = Cost::template eval<R>(d.Da, d.Db, a.W, a.H, a.ns > 0 ? a.ns : a.n, x, y, fx, fy);
        cnt = 1;
        if (e < c0) {
          d.cost[k] = e;
          d.flow[k] = ffk::pack_flow(fx, fy);
        }
      }
    }
  }
  ffk::wave_count_add(d.n_evals, cnt);
  ffk::wave_count_add2(d.n_work, cnt);
}


// Seed rerank (Eq. 1, Eq. 4): of the l ranked candidates of cell m, the one
// with the lowest E_nc, the earlier rank on equal cost; written to nn_key in
// launch_nn's relative form for the initialisation.  Counts the candidates
// but the winner (the initialisation evaluates the winner again).
struct CandPtrs {
  const uint64_t *cand[ffh::kMaxDirs];
};

template <int R, class Cost>
__global__ __launch_bounds__(256) void k_rerank(ffh::LevelArgs a, CandPtrs c, int l) {
  const ffh::LevelDir d = a.dir[blockIdx.z];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (m < a.Wn * a.Hn) {
    const int i = m % a.Wn, j = m / a.Wn;
    const int x = i * a.n, y = j * a.n;
    const uint4 qa = reinterpret_cast<const uint4 *>(d.Dq1)[(size_t)y * a.W + x];
    const uint32_t w[4] = {qa.x, qa.y, qa.z, qa.w};
    int na = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int e = (int)((w[k] >> (8 * b)) & 0xFF) - 128;
        na += e * e;
      }
    const uint64_t *cm = c.cand[blockIdx.z] + (size_t)m * l;
    uint64_t bk = ~0ull;
    uint32_t bc = 0;
    for (int k = 0; k < l; ++k) {
      const uint64_t key = cm[k];
      if (key == ~0ull) continue;
      const uint32_t q = (uint32_t)key;
      const int fx = ((int)(q % (uint32_t)a.W) - x) * (1 << Cost::kSub);
      const int fy = ((int)(q / (uint32_t)a.W) - y) * (1 << Cost::kSub);
      const uint32_t e = Cost::template eval<R>(d.Da, d.Db, a.W, a.H, a.ns > 0 ? a.ns : a.n, x, y, fx, fy);
      ++cnt;
      if (bk == ~0ull || e < bc) {
        bc = e;
        bk = key;
      }
    }
    if (bk != ~0ull)
      const_cast<uint64_t *>(d.nn_key)[m] =
          ((uint64_t)(uint32_t)((int)(bk >> 32) - na + (1 << 20)) << 32) | (uint32_t)bk;
  }
  ffk::wave_sum_add(d.n_evals, cnt > 0 ? cnt - 1 : 0);
  ffk::wave_sum_add2(d.n_work, cnt);
}

// Patch-scale change on one grid (sub-scales, Sec. 3.3): every set cell
// keeps its flow and evaluates its cost at patch scale a.ns.
template <int R, class Cost>
__global__ __launch_bounds__(256) void k_rescore(ffh::LevelArgs a) {
  const ffh::LevelDir d = a.dir[blockIdx.z];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (m < a.Wn * a.Hn && d.cost[m] != kUnset) {
    const int32_t f = d.flow[m];
    d.cost[m] = Cost::template eval<R>(d.Da, d.Db, a.W, a.H, a.ns > 0 ? a.ns : a.n, (m % a.Wn) * a.n,
                                       (m / a.Wn) * a.n, ffk::flow_x(f), ffk::flow_y(f));
    cnt = 1;
  }
  ffk::wave_count_add(d.n_evals, cnt);
  ffk::wave_count_add2(d.n_work, cnt);
}

// One propagation step in the serial order of its direction (Sec. 3.1: a
// cell after its horizontal and vertical source cells).  A cell depends only
// on its two sources, so the cells of one anti-diagonal of the scan can be
// updated together once the previous anti-diagonal is final: the grid is cut
// into kRasterTile^2 tiles, one launch handles the tiles of one tile
// anti-diagonal, and inside a tile a workgroup sweeps the cell
// anti-diagonals through LDS.  The tile's row and column before it (in scan
// order) come from tiles of earlier launches.  Per cell 16 lanes: 8 sum the
// horizontal candidate's patch terms and 8 the vertical one's; the leader
// lane applies the update of k_prop_half in serial order.
constexpr int kRasterTile = 32;
constexpr int kRasterLanes = 8;

template <int R, class Cost>
__global__ __launch_bounds__(2 * kRasterTile * kRasterLanes) void k_prop_raster(ffh::LevelArgs a, int diag,
                                                                                  int nty) {
  constexpr int S = kRasterTile, G = kRasterLanes, S1 = S + 1;
  __shared__ int32_t sf[S1 * S1];
  __shared__ uint32_t sc[S1 * S1];
  const ffh::LevelDir d = a.dir[blockIdx.z];
  const int Wn = a.Wn, Hn = a.Hn, W = a.W, H = a.H, n = a.n, ns = a.ns > 0 ? a.ns : a.n;
  const int dir = a.pass & 3;
  const int hdi = (dir == 0 || dir == 3) ? -1 : 1;
  const int vdj = (dir == 0 || dir == 2) ? -1 : 1;
  // tile (ta, tb) in scan coordinates; scan cell (sa, sb) is grid cell
  // (sa, sb) mirrored along the axes whose source lies on the high side
  const int ta = max(0, diag - (nty - 1)) + (int)blockIdx.x, tb = diag - ta;
  const int a0 = ta * S, b0 = tb * S;
  const int tw = min(S, Wn - a0), th = min(S, Hn - b0);
  auto grid_index = [&](int sa, int sb) {
    const int i = hdi < 0 ? sa : Wn - 1 - sa, j = vdj < 0 ? sb : Hn - 1 - sb;
    return j * Wn + i;
  };
  for (int e = threadIdx.x; e < (th + 1) * (tw + 1); e += blockDim.x) {
    const int lb = e / (tw + 1) - 1, la = e % (tw + 1) - 1;  // -1: the row / column before the tile
    const int sa = a0 + la, sb = b0 + lb;
    int32_t f = 0;
    uint32_t c = kUnset;  // outside the grid: no source
    if (sa >= 0 && sb >= 0) {
      const int k = grid_index(sa, sb);
      f = d.flow[k];
      c = d.cost[k];
    }
    sf[(lb + 1) * S1 + la + 1] = f;
    sc[(lb + 1) * S1 + la + 1] = c;
  }
  __syncthreads();
  const int slot = threadIdx.x / (2 * G), cand = (threadIdx.x / G) & 1, g = threadIdx.x % G;
  int cnt = 0, work = 0;
  for (int dd = 0; dd <= tw + th - 2; ++dd) {  // cell anti-diagonals of the tile
    const int amin = max(0, dd - (th - 1)), amax = min(dd, tw - 1);
    const int la = amin + slot, lb = dd - la;
    if (la <= amax) {  // uniform over the cell's 2G lanes
      const int o = (lb + 1) * S1 + la + 1;
      const int32_t f0 = sf[o], fh = sf[o - 1], fv = sf[o - S1];
      const uint32_t c0 = sc[o], ch = sc[o - 1], cv = sc[o - S1];
      const int sa = a0 + la, sb = b0 + lb;
      const int x = (hdi < 0 ? sa : Wn - 1 - sa) * n, y = (vdj < 0 ? sb : Hn - 1 - sb) * n;
      const bool set0 = c0 != kUnset;
      const bool hv = ch != kUnset && !(set0 && fh == f0) &&
                      ffk::target_in<Cost::kSub>(W, H, x, y, ffk::flow_x(fh), ffk::flow_y(fh));
      const bool vb = cv != kUnset && ffk::target_in<Cost::kSub>(W, H, x, y, ffk::flow_x(fv), ffk::flow_y(fv));
      // E(p, fv) is computed unless it is E(p, fh); whether it is used
      // depends on the horizontal outcome (the held-flow rule)
      const bool vcomp = vb && !(hv && fv == fh);
      const int32_t fc = cand == 0 ? fh : fv;
      uint32_t part = 0;
      if (cand == 0 ? hv : vcomp)
        part = Cost::template eval_part<R, G>(d.Da, d.Db, W, H, ns, x, y, ffk::flow_x(fc), ffk::flow_y(fc), g);
#pragma unroll
      for (int off = 1; off < G; off <<= 1) part += __shfl_xor(part, off);
      const uint32_t other = __shfl_xor(part, G);
      if (cand == 0 && g == 0) {
        const uint32_t eh = part, ev = other;
        uint32_t bc = c0;
        int32_t bf = f0;
        if (hv) {
          ++cnt;
          if (eh < bc) {
            bc = eh;
            bf = fh;
          }
        }
        if (vb && (bc == kUnset || fv != bf)) {
          ++cnt;
          const uint32_t e = (hv && fv == fh) ? eh : ev;
          if (e < bc) {
            bc = e;
            bf = fv;
          }
        }
        work += (int)hv + (int)vcomp;
        sf[o] = bf;
        sc[o] = bc;
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < th * tw; e += blockDim.x) {
    const int lb = e / tw, la = e % tw;
    const int k = grid_index(a0 + la, b0 + lb);
    d.flow[k] = sf[(lb + 1) * S1 + la + 1];
    d.cost[k] = sc[(lb + 1) * S1 + la + 1];
  }
  ffk::wave_sum_add(d.n_evals, cnt);
  ffk::wave_sum_add2(d.n_work, work);
}

// blockIdx.z = 1 runs the check with the roles of the two fields swapped
// (the mask of field b), in the same launch.
// Flows in units of 1/2^sb pixel: q is the pixel nearest to the target
// (halves rounded up); eps2 is the squared threshold in those units.
__global__ __launch_bounds__(256) void k_consistency(const int32_t *fa0, const uint32_t *ca0, const int32_t *fb0,
                                                     const uint32_t *cb0, int W, int H, int sb, double eps2,
                                                     uint8_t *keep_a, uint8_t *keep_b) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const bool swap = blockIdx.z == 1;
  const int32_t *fa = swap ? fb0 : fa0, *fb = swap ? fa0 : fb0;
  const uint32_t *ca = swap ? cb0 : ca0, *cb = swap ? ca0 : cb0;
  uint8_t *keep = swap ? keep_b : keep_a;
  const size_t k = (size_t)y * W + x;
  uint8_t out = 0;
  if (ca[k] != kUnset) {
    const int32_t f = fa[k];
    const int half = (1 << sb) >> 1;
    const int tx = (x << sb) + ffk::flow_x(f) + half, ty = (y << sb) + ffk::flow_y(f) + half;
    const int qx = tx >= 0 ? tx >> sb : -1, qy = ty >= 0 ? ty >> sb : -1;
    const size_t kq = (size_t)qy * W + qx;
    // fields made by the method never point outside; caller-made ones may
    if (qx >= 0 && qx < W && qy >= 0 && qy < H && cb[kq] != kUnset) {
      const int32_t g = fb[kq];
      const int64_t dx = ffk::flow_x(f) + ffk::flow_x(g), dy = ffk::flow_y(f) + ffk::flow_y(g);
      out = (double)(dx * dx + dy * dy) < eps2;
    }
  }
  keep[k] = out;
}

// The check on fields of the grid of scale n (one match per n x n region,
// Flow Fields+ Fast x2): cell (i, j) is pixel (i n, j n); the backward match
// of its target t is that of the region holding t, cell (t.x / n, t.y / n).
// blockIdx.z = 1: roles swapped (the mask of field b).
__global__ __launch_bounds__(256) void k_consistency_grid(const int32_t *fa0, const uint32_t *ca0,
                                                          const int32_t *fb0, const uint32_t *cb0, int W, int H,
                                                          int n, double eps2, uint8_t *keep_a, uint8_t *keep_b) {
  const int Wn = (W + n - 1) / n, Hn = (H + n - 1) / n;
  const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
  if (i >= Wn || j >= Hn) return;
  const bool swap = blockIdx.z == 1;
  const int32_t *fa = swap ? fb0 : fa0, *fb = swap ? fa0 : fb0;
  const uint32_t *ca = swap ? cb0 : ca0, *cb = swap ? ca0 : cb0;
  uint8_t *keep = swap ? keep_b : keep_a;
  const size_t k = (size_t)j * Wn + i;
  uint8_t out = 0;
  if (ca[k] != kUnset) {
    const int32_t f = fa[k];
    const int tx = i * n + ffk::flow_x(f), ty = j * n + ffk::flow_y(f);
    if (tx >= 0 && tx < W && ty >= 0 && ty < H) {
      const size_t kq = (size_t)(ty / n) * Wn + (size_t)(tx / n);
      if (cb[kq] != kUnset) {
        const int32_t g = fb[kq];
        const int64_t dx = ffk::flow_x(f) + ffk::flow_x(g), dy = ffk::flow_y(f) + ffk::flow_y(g);
        out = (double)(dx * dx + dy * dy) < eps2;
      }
    }
  }
  keep[k] = out;
}

// Against two backward fields (Sec. 3.7): kept iff the check above passes
// for both (their generator seeds, and possibly patch radii, differ).
__global__ __launch_bounds__(256) void k_consistency2(const int32_t *fa, const uint32_t *ca, const int32_t *fb1,
                                                      const uint32_t *cb1, const int32_t *fb2, const uint32_t *cb2,
                                                      int W, int H, double eps2, uint8_t *keep) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= W || y >= H) return;
  const size_t k = (size_t)y * W + x;
  uint8_t out = 0;
  if (ca[k] != kUnset) {
    const int32_t f = fa[k];
    const int qx = x + ffk::flow_x(f), qy = y + ffk::flow_y(f);
    const size_t kq = (size_t)qy * W + qx;
    if (qx >= 0 && qx < W && qy >= 0 && qy < H && cb1[kq] != kUnset && cb2[kq] != kUnset) {
      const int32_t g1 = fb1[kq], g2 = fb2[kq];
      const int64_t dx1 = ffk::flow_x(f) + ffk::flow_x(g1), dy1 = ffk::flow_y(f) + ffk::flow_y(g1);
      const int64_t dx2 = ffk::flow_x(f) + ffk::flow_x(g2), dy2 = ffk::flow_y(f) + ffk::flow_y(g2);
      out = (double)(dx1 * dx1 + dy1 * dy1) < eps2 && (double)(dx2 * dx2 + dy2 * dy2) < eps2;
    }
  }
  keep[k] = out;
}

// Sparsification (Sec. 3.8): one lane per q x q region; among the region's
// kept samples whose target lies in the image, the least summed consistency
// error |F_a + F_b1| (+ |F_a + F_b2|) in double precision, ties to the
// smallest pixel index (row-major scan, strict <); -1 if fewer than e kept.
__global__ __launch_bounds__(256) void k_sparsify(const int32_t *fa, const uint8_t *keep, const int32_t *fb1,
                                                  const int32_t *fb2, int W, int H, int q, int e, int32_t *sel) {
  const int Wq = (W + q - 1) / q, Hq = (H + q - 1) / q;
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (long long)Wq * Hq) return;
  const int rx = (int)(r % Wq), ry = (int)(r / Wq);
  int count = 0, best = -1;
  double best_err = 0.0;
  for (int y = ry * q; y < min(ry * q + q, H); ++y)
    for (int x = rx * q; x < min(rx * q + q, W); ++x) {
      const size_t k = (size_t)y * W + x;
      if (!keep[k]) continue;
      ++count;
      const int32_t f = fa[k];
      const int tx = x + ffk::flow_x(f), ty = y + ffk::flow_y(f);
      if (tx < 0 || tx >= W || ty < 0 || ty >= H) continue;
      const size_t kt = (size_t)ty * W + tx;
      const int32_t g1 = fb1[kt];
      const double dx = ffk::flow_x(f) + ffk::flow_x(g1), dy = ffk::flow_y(f) + ffk::flow_y(g1);
      double err = sqrt(dx * dx + dy * dy);
      if (fb2) {
        const int32_t g2 = fb2[kt];
        const double ex = ffk::flow_x(f) + ffk::flow_x(g2), ey = ffk::flow_y(f) + ffk::flow_y(g2);
        err += sqrt(ex * ex + ey * ey);
      }
      if (best < 0 || err < best_err) {
        best = (int)k;
        best_err = err;
      }
    }
  sel[r] = count >= e ? best : -1;
}

// Batches: items = (pair, direction, row); direction 1 writes the backward
// mask when the pair has one.
__global__ __launch_bounds__(256) void k_consistency_batch(ffh::BatchStage st, double eps2) {
  ffk::for_items(st.total, [&](int item) {
    const int p = ffk::batch_pair(st.prefix, st.npairs, item);
    const ffh::BatchPair &bp = st.pairs[p];
    const int local = item - st.prefix[p];
    const int dir = local / bp.H, y = local % bp.H, W = bp.W, H = bp.H;
    uint8_t *keep = bp.keep[dir];
    if (keep == nullptr) return;
    const int32_t *fa = bp.gflow[0][dir], *fb = bp.gflow[0][dir ^ 1];
    const uint32_t *ca = bp.gcost[0][dir], *cb = bp.gcost[0][dir ^ 1];
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
      const size_t k = (size_t)y * W + x;
      uint8_t out = 0;
      if (ca[k] != kUnset) {
        const int32_t f = fa[k];
        const int qx = x + ffk::flow_x(f), qy = y + ffk::flow_y(f);
        const size_t kq = (size_t)qy * W + qx;
        if (qx >= 0 && qx < W && qy >= 0 && qy < H && cb[kq] != kUnset) {
          const int32_t g = fb[kq];
          const int64_t dx = ffk::flow_x(f) + ffk::flow_x(g), dy = ffk::flow_y(f) + ffk::flow_y(g);
          out = (double)(dx * dx + dy * dy) < eps2;
        }
      }
      keep[k] = out;
    }
  });
}

#define FF_RADIUS_SWITCH_C(R_, CALL, C_)                                        \
  switch (R_) {                                                                 \
    case 0: CALL(0, C_); break;                                                 \
    case 1: CALL(1, C_); break;                                                 \
    case 2: CALL(2, C_); break;                                                 \
    case 3: CALL(3, C_); break;                                                 \
    case 4: CALL(4, C_); break;                                                 \
    case 5: CALL(5, C_); break;                                                 \
    case 6: CALL(6, C_); break;                                                 \
    case 7: CALL(7, C_); break;                                                 \
    default: return hipErrorInvalidValue;                                       \
  }
#define FF_RADIUS_SWITCH(A_, CALL)                                              \
  if ((A_).fcost == 1) {                                                        \
    FF_RADIUS_SWITCH_C((A_).radius, CALL, ffk::CostF32)                         \
  } else if ((A_).fcost == 2) {                                                 \
    FF_RADIUS_SWITCH_C((A_).radius, CALL, ffk::CostU8Sub)                       \
  } else {                                                                      \
    FF_RADIUS_SWITCH_C((A_).radius, CALL, ffk::CostU8)                          \
  }

}  // namespace

namespace ffh {

hipError_t launch_init_coarse(const LevelArgs &a, hipStream_t stream) {
  const int cells = a.Wn * a.Hn;
  dim3 grid((cells + 255) / 256, 1, a.ndir);
#define CALL(R, C) hipLaunchKernelGGL((k_init_coarse<R, C>), grid, dim3(256), 0, stream, a)
  FF_RADIUS_SWITCH(a, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_seed_level(const LevelArgs &a, hipStream_t stream) {
  const int cells = a.Wn * a.Hn;
  dim3 grid((cells + 255) / 256, 1, a.ndir);
#define CALL(R, C) hipLaunchKernelGGL((k_seed_level<R, C>), grid, dim3(256), 0, stream, a)
  FF_RADIUS_SWITCH(a, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_propagate(const LevelArgs &a, hipStream_t stream) {
  const int half = (a.Wn + 1) / 2;
  dim3 grid((half + 63) / 64, (a.Hn + 3) / 4, a.ndir);
  for (int colour = 1; colour >= 0; --colour) {
#define CALL(R, C) hipLaunchKernelGGL((k_prop_half<R, C>), grid, dim3(256), 0, stream, a, colour)
    FF_RADIUS_SWITCH(a, CALL)
#undef CALL
  }
  return hipGetLastError();
}

hipError_t launch_rerank(const LevelArgs &a, const uint64_t *const *cand, int l, hipStream_t stream) {
  if (l < 1 || l > kTopLMax) return hipErrorInvalidValue;
  CandPtrs c{};
  for (int dr = 0; dr < a.ndir; ++dr) c.cand[dr] = cand[dr];
  const int cells = a.Wn * a.Hn;
  dim3 grid((cells + 255) / 256, 1, a.ndir);
#define CALL(R, C) hipLaunchKernelGGL((k_rerank<R, C>), grid, dim3(256), 0, stream, a, c, l)
  FF_RADIUS_SWITCH(a, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_rescore(const LevelArgs &a, hipStream_t stream) {
  const int cells = a.Wn * a.Hn;
  dim3 grid((cells + 255) / 256, 1, a.ndir);
#define CALL(R, C) hipLaunchKernelGGL((k_rescore<R, C>), grid, dim3(256), 0, stream, a)
  FF_RADIUS_SWITCH(a, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_propagate_raster(const LevelArgs &a, hipStream_t stream) {
  const int ntx = (a.Wn + kRasterTile - 1) / kRasterTile, nty = (a.Hn + kRasterTile - 1) / kRasterTile;
  for (int diag = 0; diag < ntx + nty - 1; ++diag) {
    const int lo = std::max(0, diag - (nty - 1)), hi = std::min(diag, ntx - 1);
    dim3 grid(hi - lo + 1, 1, a.ndir);
#define CALL(R, C) hipLaunchKernelGGL((k_prop_raster<R, C>), grid, dim3(2 * kRasterTile * kRasterLanes), 0, stream, a, diag, nty)
    if (a.fcost == 2) {
      FF_RADIUS_SWITCH_C(a.radius, CALL, ffk::CostU8Sub)
    } else if (a.fcost == 0) {
      FF_RADIUS_SWITCH_C(a.radius, CALL, ffk::CostU8)
    } else {
      return hipErrorInvalidValue;  // integer costs only
    }
#undef CALL
  }
  return hipGetLastError();
}

hipError_t launch_random_search(const LevelArgs &a, hipStream_t stream) {
  dim3 grid((a.Wn + 63) / 64, (a.Hn + 3) / 4, a.ndir);
#define CALL(R, C) hipLaunchKernelGGL((k_random_search<R, C>), grid, dim3(256), 0, stream, a)
  FF_RADIUS_SWITCH(a, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_batch_consistency(const BatchStage &rows, float eps, hipStream_t stream) {
  if (rows.total <= 0) return hipSuccess;
  const dim3 grid(((std::min(rows.total, 4096) + 7) / 8) * 8);
  hipLaunchKernelGGL(k_consistency_batch, grid, dim3(256), 0, stream, rows, (double)eps * (double)eps);
  return hipGetLastError();
}

hipError_t launch_sparsify(const int16_t *fa, const uint8_t *keep, const int16_t *fb1, const int16_t *fb2, int W,
                           int H, int q, int e, int32_t *sel, hipStream_t stream) {
  const long long regions = (long long)((W + q - 1) / q) * ((H + q - 1) / q);
  hipLaunchKernelGGL(k_sparsify, dim3((unsigned)((regions + 255) / 256)), dim3(256), 0, stream,
                     reinterpret_cast<const int32_t *>(fa), keep, reinterpret_cast<const int32_t *>(fb1),
                     reinterpret_cast<const int32_t *>(fb2), W, H, q, e, sel);
  return hipGetLastError();
}

hipError_t launch_consistency2(const int16_t *fa, const uint32_t *ca, const int16_t *fb1, const uint32_t *cb1,
                               const int16_t *fb2, const uint32_t *cb2, int W, int H, float eps, uint8_t *keep,
                               hipStream_t stream) {
  dim3 grid((W + 255) / 256, H);
  const double eps2 = (double)eps * (double)eps;
  hipLaunchKernelGGL(k_consistency2, grid, dim3(256), 0, stream, reinterpret_cast<const int32_t *>(fa), ca,
                     reinterpret_cast<const int32_t *>(fb1), cb1, reinterpret_cast<const int32_t *>(fb2), cb2, W, H,
                     eps2, keep);
  return hipGetLastError();
}

hipError_t launch_consistency_grid(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb,
                                  int W, int H, int n, float eps, uint8_t *keep_a, uint8_t *keep_b,
                                  hipStream_t stream) {
  const int Wn = (W + n - 1) / n, Hn = (H + n - 1) / n;
  dim3 grid((Wn + 255) / 256, Hn, keep_b ? 2 : 1);
  hipLaunchKernelGGL(k_consistency_grid, grid, dim3(256), 0, stream, reinterpret_cast<const int32_t *>(fa), ca,
                     reinterpret_cast<const int32_t *>(fb), cb, W, H, n, (double)eps * (double)eps, keep_a, keep_b);
  return hipGetLastError();
}

hipError_t launch_consistency(const int16_t *fa, const uint32_t *ca, const int16_t *fb, const uint32_t *cb, int W,
                              int H, float eps, uint8_t *keep_a, uint8_t *keep_b, hipStream_t stream, int sb) {
  dim3 grid((W + 255) / 256, H, keep_b ? 2 : 1);
  const double lim = (double)eps * (double)(1 << sb);
  hipLaunchKernelGGL(k_consistency, grid, dim3(256), 0, stream, reinterpret_cast<const int32_t *>(fa), ca,
                     reinterpret_cast<const int32_t *>(fb), cb, W, H, sb, lim * lim, keep_a, keep_b);
  return hipGetLastError();
}

}  // namespace ffh
