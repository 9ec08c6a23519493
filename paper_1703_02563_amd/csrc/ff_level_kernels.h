// Kernels and launchers of the temporally blocked level kernel; included by
// the per-scale translation units ff_level_s*.hip (each instantiates the
// kernels of one scale, so that they compile in parallel).
//
// Temporally blocked level kernel: a run of propagation steps (Eq. 2) and
// random-search steps (Sec. 3.1) of one scale in one launch (Sec. 3.2
// schedule), for patch radius 3.
//
// Each workgroup owns a TW x TH tile of the level grid and keeps the flow
// and cost of the tile plus a halo in LDS.  A half-sweep that reads sources
// on one side can only update correctly the cells whose source lies inside
// the currently valid window, so the valid window loses one cell on every
// side the half-sweep reads from.  The halo of a run equals the number of
// half-sweeps that read each side, so after the last step exactly the owned
// tile is valid and is written back.  Cells of the halo are computed
// redundantly by the neighbouring workgroups; evaluations are counted only
// for owned cells, so the count equals the unblocked schedule's.
//
// The scale-n descriptors of image a are staged in LDS on the level
// lattice (virtual cell (i+u, j+v) -> pixel clamp((i+u)n, (j+v)n)), which is
// exactly where E_n reads them.  Image b is read at p + f + n(u, v) with f
// per cell, straight from global memory.  The descriptor maps are padded
// with a replicated border of 3n pixels and their rows are in phase order,
// so every patch read is unclamped and contiguous at every scale.
//
// A half-sweep checks every cell's sources and queues the evaluations that
// can matter, evaluates the queue densely (one lane, or a quad of lanes, per
// evaluation) and then decodes each cell's best candidate; a random-search
// step evaluates one queued candidate per cell.
#pragma once

#include <algorithm>
#include <type_traits>

#include "ff_device.h"
#include "ff_internal.h"

namespace {

using ffk::clampi;
using ffk::kUnset;

constexpr int kR = 3;
constexpr int kHalo = ffh::kLevelHalo;

template <int TW, int TH, int HALO = kHalo, int RR = kR>
struct Geo {
  static constexpr int LW = TW + 2 * HALO, LH = TH + 2 * HALO;  // state window
  static constexpr int DW = LW + 2 * RR, DH = LH + 2 * RR;        // descriptor window (patch radius RR)
  static_assert(2 * LW * LH < 65536, "queue entries are 16-bit: cell * 2 + vertical");
};

// E_n(p, f) with image-a descriptors from LDS.  `pa` points at the LDS
// descriptor of the cell itself; (bx, by) = p + f in pixels, inside the
// image, so the whole patch lies in the padded map of image b: no clamps,
// and the samples of a patch row are consecutive stored columns (phase
// order) loaded with immediate offsets.  EV selects the load schedule:
// 0 rows one after another, 1 rows unrolled (the compiler interleaves),
// 2 all 49 loads issued before any arithmetic (needs ~200 registers); EV 3
// evaluates with a quad of lanes instead (eval_quad).
template <int LOG2N, int DW, int EV, int RR = kR>
__device__ __forceinline__ uint32_t eval_cell(const uint4 *pa, const uint4 *__restrict__ Db, int W, int bx, int by) {
  constexpr int n = 1 << LOG2N, P = ffk::kDescPad * n, K = 2 * RR + 1;
  const int Wp = W + 2 * P;
  uint32_t s = 0;
  const uint4 *pb = Db + ffk::desc_index(bx - RR * n, by - RR * n, LOG2N, W);
  if constexpr (EV == 2) {
    uint4 b[K * K];
#pragma unroll
    for (int v = 0; v < K; ++v)
#pragma unroll
      for (int u = 0; u < K; ++u) b[v * K + u] = pb[(size_t)v * n * Wp + u];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < K; ++v) {
      const uint4 *ra = pa + (v - RR) * DW - RR;
#pragma unroll
      for (int u = 0; u < K; ++u) s = ffk::sad16(ra[u], b[v * K + u], s);
    }
  } else {
#pragma unroll EV ? K : 1
    for (int v = 0; v < K; ++v) {
      const uint4 *ra = pa + (v - RR) * DW - RR;
#pragma unroll
      for (int u = 0; u < K; ++u) s = ffk::sad16(ra[u], pb[u], s);
      pb += (size_t)n * Wp;
    }
  }
  return s;
}

// E_n(p, f) evaluated by the four lanes of a quad (lanes 4k .. 4k+3 of a
// wave, all active): lane r takes patch columns u = r and u = r + 4 (none for
// r = 3) of all seven rows, so one load instruction of a quad covers four
// consecutive samples (64 contiguous bytes of a patch row) instead of one
// sample per lane spread over 64 patches.  Image b is read through a buffer
// resource over its padded map (the row offset rides in the scalar offset);
// the partial sums are added across the quad, every lane returns the total.
// Requires a map of less than 2^31 bytes.
// E_n(p, f) of a radius-4 patch (9 x 9) by a quad: lane r takes columns
// r, r + 4 and r + 8 (the last for lane 0 only), one column after another.
template <int LOG2N, int DW>
__device__ __forceinline__ uint32_t eval_quad9(const uint4 *pa, __amdgpu_buffer_rsrc_t db, int W, int bx, int by,
                                               int r) {
  constexpr int n = 1 << LOG2N, P = ffk::kDescPad * n, RR = 4, K = 2 * RR + 1;
  const int rowb = n * (W + 2 * P) * 16;
  const int off = (int)ffk::desc_index(bx - RR * n, by - RR * n, LOG2N, W) * 16;
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int u = min(r + 4 * c, K - 1);
    uint4 b[K];
#pragma unroll
    for (int v = 0; v < K; ++v) {
      const auto x = __builtin_amdgcn_raw_buffer_load_b128(db, off + u * 16, v * rowb, 0);
      b[v] = make_uint4(x[0], x[1], x[2], x[3]);
    }
    const uint4 *ra = pa - RR * DW - RR + u;
    uint32_t t = 0;
#pragma unroll
    for (int v = 0; v < K; ++v) t = ffk::sad16(ra[v * DW], b[v], t);
    s += (r + 4 * c < K) ? t : 0u;
  }
  s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  return s;
}

template <int LOG2N, int DW, int RR = kR>
__device__ __forceinline__ uint32_t eval_quad(const uint4 *pa, __amdgpu_buffer_rsrc_t db, int W, int bx, int by,
                                              int r) {
  if constexpr (RR == 4) {
    return eval_quad9<LOG2N, DW>(pa, db, W, bx, by, r);
  } else {
    constexpr int n = 1 << LOG2N, P = ffk::kDescPad * n, K = 2 * RR + 1;
    const int rowb = n * (W + 2 * P) * 16;
    const int u1 = r, u2 = min(r + 4, K - 1);
    const int off = (int)ffk::desc_index(bx - RR * n, by - RR * n, LOG2N, W) * 16;
    uint4 b1[K], b2[K], a1[K], a2[K];
#pragma unroll
    for (int v = 0; v < K; ++v) {
      const auto x = __builtin_amdgcn_raw_buffer_load_b128(db, off + u1 * 16, v * rowb, 0);
      const auto y = __builtin_amdgcn_raw_buffer_load_b128(db, off + u2 * 16, v * rowb, 0);
      b1[v] = make_uint4(x[0], x[1], x[2], x[3]);
      b2[v] = make_uint4(y[0], y[1], y[2], y[3]);
    }
    // image a's samples from LDS while the global loads are in flight: the
    // first column's now, the second's once half of the first is summed (so
    // that fewer than 128 registers hold the whole evaluation)
    const uint4 *ra1 = pa - RR * DW - RR + u1, *ra2 = pa - RR * DW - RR + u2;
#pragma unroll
    for (int v = 0; v < K; ++v) a1[v] = ra1[v * DW];
    __builtin_amdgcn_sched_barrier(0);
    uint32_t s1 = 0, s2 = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) s1 = ffk::sad16(a1[v], b1[v], s1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 0; v < K; ++v) a2[v] = ra2[v * DW];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int v = 4; v < K; ++v) s1 = ffk::sad16(a1[v], b1[v], s1);
#pragma unroll
    for (int v = 0; v < K; ++v) s2 = ffk::sad16(a2[v], b2[v], s2);
    uint32_t s = s1 + (r < K - 4 ? s2 : 0u);
    s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    return s;
}
}
// The same with image a's patch also read from its padded map (a quad per
// evaluation; the cells the weight-class evaluation does not cover).
template <int LOG2N, int RR = kR>
__device__ __forceinline__ uint32_t eval_quad_gg(__amdgpu_buffer_rsrc_t da, __amdgpu_buffer_rsrc_t db, int W, int ax,
                                                 int ay, int bx, int by, int r) {
  constexpr int n = 1 << LOG2N, P = ffk::kDescPad * n, K = 2 * RR + 1;
  const int rowb = n * (W + 2 * P) * 16;
  const int u1 = r, u2 = min(r + 4, K - 1);
  const int offa = (int)ffk::desc_index(ax - RR * n, ay - RR * n, LOG2N, W) * 16;
  const int offb = (int)ffk::desc_index(bx - RR * n, by - RR * n, LOG2N, W) * 16;
  uint32_t s1 = 0, s2 = 0;
#pragma unroll
  for (int v = 0; v < K; ++v) {
    const auto a1 = __builtin_amdgcn_raw_buffer_load_b128(da, offa + u1 * 16, v * rowb, 0);
    const auto a2 = __builtin_amdgcn_raw_buffer_load_b128(da, offa + u2 * 16, v * rowb, 0);
    const auto b1 = __builtin_amdgcn_raw_buffer_load_b128(db, offb + u1 * 16, v * rowb, 0);
    const auto b2 = __builtin_amdgcn_raw_buffer_load_b128(db, offb + u2 * 16, v * rowb, 0);
    s1 = ffk::sad16(make_uint4(a1[0], a1[1], a1[2], a1[3]), make_uint4(b1[0], b1[1], b1[2], b1[3]), s1);
    s2 = ffk::sad16(make_uint4(a2[0], a2[1], a2[2], a2[3]), make_uint4(b2[0], b2[1], b2[2], b2[3]), s2);
  }
  uint32_t s = s1 + (r < K - 4 ? s2 : 0u);
  s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  return s;
}

// E(p, f) at the patch scale m of a sub-scale stage (Sec. 3.3) by a quad,
// both images read from their image-order maps of scale m (border
// P = kDescPad * m, rows of W + 2P entries; a sample p + m (u, v) of a patch
// around an in-image pixel lies inside the border, so no clamping): lane r
// sums columns r and r + 4 of the 7 x 7 samples, the quad adds the lanes.
// Integer sums: the value is that of the per-step kernels' patch_cost.
template <int RR = kR>
__device__ __forceinline__ uint32_t eval_quad_sub(__amdgpu_buffer_rsrc_t da, __amdgpu_buffer_rsrc_t db, int W, int m,
                                                  int ax, int ay, int bx, int by, int r) {
  constexpr int K = 2 * RR + 1;
  const int P = ffk::desc_pad(m), Wp = W + 2 * P;
  const int rowb = m * Wp * 16, colb = m * 16;
  const int u1 = r, u2 = min(r + 4, K - 1);
  const int offa = ((ay - RR * m + P) * Wp + (ax - RR * m + P)) * 16;
  const int offb = ((by - RR * m + P) * Wp + (bx - RR * m + P)) * 16;
  uint32_t s1 = 0, s2 = 0;
#pragma unroll
  for (int v = 0; v < K; ++v) {
    const auto a1 = __builtin_amdgcn_raw_buffer_load_b128(da, offa + u1 * colb, v * rowb, 0);
    const auto a2 = __builtin_amdgcn_raw_buffer_load_b128(da, offa + u2 * colb, v * rowb, 0);
    const auto b1 = __builtin_amdgcn_raw_buffer_load_b128(db, offb + u1 * colb, v * rowb, 0);
    const auto b2 = __builtin_amdgcn_raw_buffer_load_b128(db, offb + u2 * colb, v * rowb, 0);
    s1 = ffk::sad16(make_uint4(a1[0], a1[1], a1[2], a1[3]), make_uint4(b1[0], b1[1], b1[2], b1[3]), s1);
    s2 = ffk::sad16(make_uint4(a2[0], a2[1], a2[2], a2[3]), make_uint4(b2[0], b2[1], b2[2], b2[3]), s2);
  }
  uint32_t s = s1 + (r < K - 4 ? s2 : 0u);
  s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  s += (uint32_t)__builtin_amdgcn_mov_dpp((int)s, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  return s;
}

// E_n(p, f) by one lane from the weight-class row maps (wform_index), for a
// cell p and a target (bx, by) both at least 3n inside the image: the 13
// rows y + n b (b = -6..6) of image a come from LDS (`pa`: the cell's entry
// of row b = -6 in a window of row length LW), those of image b from its
// map (one 16-byte load per row, the row step in the scalar offset); four
// byte SADs per row go to the accumulator of its (row weight, column
// weight) class, and E = sum_{l,k} l k T[l][k].
template <int LOG2N, int LW>
__device__ __forceinline__ uint32_t eval_wform(const uint4 *pa, __amdgpu_buffer_rsrc_t wb, int W, int bx, int by) {
  constexpr int n = 1 << LOG2N, K = 13;
  constexpr int kRowClass[K] = {0, 0, 1, 1, 2, 2, 3, 2, 2, 1, 1, 0, 0};  // w(b) - 1
  const int rowb = n * W * 16;
  const int off = (int)ffk::wform_index(bx, by - 6 * n, n, W) * 16;
  uint4 B[K];
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b128(wb, off, b * rowb, 0);
    B[b] = make_uint4(x[0], x[1], x[2], x[3]);
  }
  uint32_t T[4][4] = {};
#pragma unroll
  for (int b = 0; b < K; ++b) {
    const uint4 A = pa[b * LW];
    const int l = kRowClass[b];
    T[l][0] = __builtin_amdgcn_sad_u8(A.x, B[b].x, T[l][0]);
    T[l][1] = __builtin_amdgcn_sad_u8(A.y, B[b].y, T[l][1]);
    T[l][2] = __builtin_amdgcn_sad_u8(A.z, B[b].z, T[l][2]);
    T[l][3] = __builtin_amdgcn_sad_u8(A.w, B[b].w, T[l][3]);
  }
  uint32_t R[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) R[l] = T[l][0] + 2 * T[l][1] + 3 * T[l][2] + 4 * T[l][3];
  return R[0] + 2 * R[1] + 3 * R[2] + 4 * R[3];
}

// Float learned-feature cost (Eq. 3 with the squared-difference data term)
// by a quad of lanes: lane r owns channels 4r .. 4r+3 and sums their terms
// with one fused multiply-add each in the order v, u, c; the quad then adds
// the four partial sums as (s0 + s1) + (s2 + s3) (every lane returns the
// total, as a bit pattern).  Image a's lattice samples come from LDS (`pa`:
// the cell's 4 float4 in a window of row length DW cells), image b's from
// its padded, phase-ordered map (64-byte entries): a quad reads one whole
// entry per load.
template <int LOG2N, int DW>
__device__ __forceinline__ uint32_t eval_quad_f32(const float4 *pa, const float4 *__restrict__ B, int W, int bx,
                                                  int by, int r) {
  constexpr int n = 1 << LOG2N, P = ffk::kDescPad * n, K = 2 * kR + 1;
  const size_t row = (size_t)n * (W + 2 * P) * 4;
  const float4 *pb = B + 4 * ffk::desc_index(bx - kR * n, by - kR * n, LOG2N, W) + r;
  const float4 *ra = pa + (-kR * DW - kR) * 4 + r;
  float s = 0.0f;
#pragma unroll
  for (int v = 0; v < K; ++v) {
    float4 y[K];
#pragma unroll
    for (int u = 0; u < K; ++u) y[u] = pb[v * row + 4 * u];
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const float4 x = ra[(v * DW + u) * 4];
      float e = x.x - y[u].x;
      s = __fmaf_rn(e, e, s);
      e = x.y - y[u].y;
      s = __fmaf_rn(e, e, s);
      e = x.z - y[u].z;
      s = __fmaf_rn(e, e, s);
      e = x.w - y[u].w;
      s = __fmaf_rn(e, e, s);
    }
  }
  s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0xB1, 0xF, 0xF, false));  // quad_perm [1,0,3,2]
  s += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(s), 0x4E, 0xF, 0xF, false));  // quad_perm [2,3,0,1]
  return __float_as_uint(s);
}

// The run of passes for tile `tile` of one direction `d` (a holds the
// pair's sizes and the schedule).  All threads of the workgroup call it.
template <int LOG2N, int TW, int TH, int kThreads, int EV, bool F32 = false, int HALO = kHalo, int RR = kR,
          bool SUB = false>
__device__ __forceinline__ void level_body(const ffh::LevelKArgs &a, const ffh::LevelKDir &d, int tile) {
  // SUB: a sub-scale stage (patch scale a.sub_m, image-order maps), descriptor quads at radius 3
  static_assert(!SUB || (EV == 3 && !F32 && RR == kR), "sub-scale stages run the radius-3 quad kernels");
  // patch radius RR: 3, or 2 and 4 with the descriptor-quad evaluations
  // (the weight-class maps and the float path hold radius-3 patches)
  static_assert(Geo<TW, TH, HALO, RR>::LW * Geo<TW, TH, HALO, RR>::LH + kThreads < 65536,
                "the cell index of a half-sweep must stay below 2^16 (cell_of's division)");
  static_assert(RR == kR || ((RR == 2 || RR == 4) && EV == 3 && !F32),
                "radii 2 and 4 run the descriptor-quad kernels only");
  using G = Geo<TW, TH, HALO, RR>;
  constexpr int n = 1 << LOG2N;
  // EV 3 and float features: every evaluation by a quad of lanes
  // (eval_quad, eval_quad_f32); the candidate flows of a random-search step
  // are then parked in s_flags.  EV 4: evaluations whose cell and target lie
  // 3n inside the image by one lane each on the weight-class row maps
  // (eval_wform, image a's rows staged in LDS), the others by a quad
  // reading both descriptor maps (eval_quad_gg); such queues fill from the
  // front (weight-class) and from the back (descriptor quads).
  constexpr bool WF = EV == 4;
  constexpr bool QUAD = EV == 3 || F32 || WF;
  constexpr int QCAP = G::LH * G::LW + G::LH;
  constexpr int kQuads = kThreads / 4;
  using FlagT = std::conditional_t<QUAD, uint32_t, uint8_t>;
  __shared__ int32_t s_flow[G::LH * G::LW];
  __shared__ uint32_t s_cost[G::LH * G::LW];
  // byte descriptors of image a on the level lattice (float features are
  // read from their padded map instead); 64-bit keys for float costs
  __shared__ uint4 s_da[(F32 || WF) ? 1 : G::DH * G::DW];
  // weight-class row entries of image a: window rows gj0 - 6 ... gj0 + LH + 5
  __shared__ uint4 s_wa[WF ? (G::LH + 12) * G::LW : 1];
  __shared__ float4 s_daf[F32 ? 4 * G::DH * G::DW : 1];
  __shared__ unsigned long long s_key[F32 ? G::LH * G::LW : 1];
  __shared__ uint16_t s_queue[QCAP];  // queued evaluations: cell * 2 + vertical
  // candidate flags of the current half-sweep; with quads also the parked
  // random-search candidate flows
  __shared__ FlagT s_flags[G::LH * G::LW];
  __shared__ unsigned int s_cnt, s_qlen, s_rlen, s_blen, s_rblen;
  __shared__ unsigned int s_work[2];  // evaluations computed: owned cells, all cells

  const int tid = threadIdx.x, qr = tid & 3;
  const int W = a.W, H = a.H, Wn = a.Wn, Hn = a.Hn;
  const int ti0 = (tile % a.tiles_x) * TW, tj0 = (tile / a.tiles_x) * TH;
  const int oi1 = min(ti0 + TW, Wn), oj1 = min(tj0 + TH, Hn);
  const int gi0 = ti0 - HALO, gj0 = tj0 - HALO;  // grid coords of window cell (0, 0)
  auto owned = [&](int i, int j) { return i >= ti0 && i < oi1 && j >= tj0 && j < oj1; };
  const uint4 *Db = reinterpret_cast<const uint4 *>(d.Db);
  if (tid == 0) {
    s_cnt = 0;
    s_qlen = 0;
    s_rlen = 0;
    s_blen = 0;
    s_rblen = 0;
    s_work[0] = 0;
    s_work[1] = 0;
  }

  // image-a descriptors on the level lattice around the window: every load
  // of a thread is issued before the first LDS store (one memory round trip)
  constexpr int NSTAGE = F32 ? 4 * G::DH * G::DW : (WF ? (G::LH + 12) * G::LW : G::DH * G::DW);
  constexpr int NS = (NSTAGE + kThreads - 1) / kThreads;
  uint4 sv[F32 ? 1 : NS];
  float4 sf[F32 ? NS : 1];
  if constexpr (WF) {
    const uint4 *Wa = reinterpret_cast<const uint4 *>(d.Wa);
#pragma unroll
    for (int it = 0; it < NS; ++it) {
      const int k = min(it * kThreads + tid, NSTAGE - 1);
      const int vi = gi0 + k % G::LW, vj = gj0 - 6 + k / G::LW;
      sv[it] = Wa[ffk::wform_index(clampi(vi * n, W - 1), clampi(vj * n, H - 1), n, W)];
    }
  } else if constexpr (!F32) {
    const uint4 *Da = reinterpret_cast<const uint4 *>(d.Da);
    uint4 *v = sv;
    if constexpr (!SUB) {  // a sub-scale stage reads image a from its map instead
#pragma unroll
      for (int it = 0; it < NS; ++it) {
        const int k = min(it * kThreads + tid, G::DH * G::DW - 1);
        const int vi = gi0 - RR + k % G::DW, vj = gj0 - RR + k / G::DW;
        v[it] = Da[ffk::desc_index(clampi(vi * n, W - 1), clampi(vj * n, H - 1), LOG2N, W)];
      }
    }
  } else {
    const float4 *Da = reinterpret_cast<const float4 *>(d.Da);
    float4 *v = sf;
#pragma unroll
    for (int it = 0; it < NS; ++it) {
      const int k = min(it * kThreads + tid, 4 * G::DH * G::DW - 1);
      const int c = k >> 2, vi = gi0 - RR + c % G::DW, vj = gj0 - RR + c / G::DW;
      v[it] = Da[4 * ffk::desc_index(clampi(vi * n, W - 1), clampi(vj * n, H - 1), LOG2N, W) + (k & 3)];
    }
  }
  // E_n of grid cell (i, j) and target pixel (bx, by), one lane per
  // evaluation (byte descriptors, EV 0-2)
  auto evalc = [&](int i, int j, int bx, int by) -> uint32_t {
    const uint4 *pa = s_da + (j - gj0 + RR) * G::DW + (i - gi0 + RR);
    return eval_cell<LOG2N, G::DW, (EV < 3 ? EV : 1), RR>(pa, Db, W, bx, by);
  };
  // the same by a quad of lanes (QUAD only)
  [[maybe_unused]] const __amdgpu_buffer_rsrc_t db_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(d.Db), (short)0,
      (int)((size_t)(H + 2 * ffk::desc_pad(n)) * (W + 2 * ffk::desc_pad(n)) * 16), 0x00020000);
  auto evalq = [&](int i, int j, int bx, int by) -> uint32_t {
    if constexpr (F32) {
      const float4 *pa = s_daf + 4 * ((j - gj0 + RR) * G::DW + (i - gi0 + RR));
      return eval_quad_f32<LOG2N, G::DW>(pa, reinterpret_cast<const float4 *>(d.Db), W, bx, by, qr);
    } else if constexpr (SUB) {
      // both maps of patch scale a.sub_m (image order) through resources
      // of their size
      const int sm = a.sub_m;
      const int bytes = (int)((size_t)(H + 2 * ffk::desc_pad(sm)) * (W + 2 * ffk::desc_pad(sm)) * 16);
      const __amdgpu_buffer_rsrc_t ra =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(d.Da), (short)0, bytes, 0x00020000);
      const __amdgpu_buffer_rsrc_t rb =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(d.Db), (short)0, bytes, 0x00020000);
      return eval_quad_sub<RR>(ra, rb, W, sm, i * n, j * n, bx, by, qr);
    } else {
      const uint4 *pa = s_da + (j - gj0 + RR) * G::DW + (i - gi0 + RR);
      return eval_quad<LOG2N, G::DW, RR>(pa, db_rsrc, W, bx, by, qr);
    }
  };
  // evaluations computed (the work counters; a no-op without them), called
  // by every lane of a wave
  auto count_work = [&](bool did, bool own) {
    if (d.n_work == nullptr) return;
    const int all = __popcll(__ballot(did)), mine = __popcll(__ballot(did && own));
    if ((tid & 63) == 0 && all) {
      atomicAdd(&s_work[0], (unsigned)mine);
      atomicAdd(&s_work[1], (unsigned)all);
    }
  };
  // the weight-class path: interior test, one-lane and all-global quad evaluations
  [[maybe_unused]] const __amdgpu_buffer_rsrc_t wb_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(d.Wb), (short)0, WF ? (int)ffk::wform_bytes(W, H, n) : 0, 0x00020000);
  [[maybe_unused]] const __amdgpu_buffer_rsrc_t da_rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<uint8_t *>(d.Da), (short)0,
      WF ? (int)((size_t)(H + 2 * ffk::desc_pad(n)) * (W + 2 * ffk::desc_pad(n)) * 16) : 0, 0x00020000);
  [[maybe_unused]] auto inner = [&](int i, int j, int bx, int by) {
    const int lo = 3 * n;
    return i * n >= lo && i * n <= W - 1 - lo && j * n >= lo && j * n <= H - 1 - lo && bx >= lo && bx <= W - 1 - lo &&
           by >= lo && by <= H - 1 - lo;
  };
  [[maybe_unused]] auto evalw = [&](int i, int j, int bx, int by) -> uint32_t {
    return eval_wform<LOG2N, G::LW>(s_wa + (j - gj0) * G::LW + (i - gi0), wb_rsrc, W, bx, by);
  };
  [[maybe_unused]] auto evalg = [&](int i, int j, int bx, int by) -> uint32_t {
    return eval_quad_gg<LOG2N, RR>(da_rsrc, db_rsrc, W, i * n, j * n, bx, by, qr);
  };
  // append of the lanes with `on` set, at the front (inn) or the back (!inn)
  // of the queue: one LDS atomic per wave and end
  [[maybe_unused]] auto enqueue2 = [&](bool on, bool inn, uint16_t e, unsigned int &flen, unsigned int &blen) {
    const uint64_t bi = __ballot(on && inn), bb = __ballot(on && !inn);
    int q0 = 0, q1 = 0;
    if ((tid & 63) == 0) {
      if (bi) q0 = (int)atomicAdd(&flen, (unsigned)__popcll(bi));
      if (bb) q1 = (int)atomicAdd(&blen, (unsigned)__popcll(bb));
    }
    q0 = __shfl(q0, 0);
    q1 = __shfl(q1, 0);
    const int lane = tid & 63;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (on && inn) s_queue[q0 + __popcll(bi & below)] = e;
    if (on && !inn) s_queue[QCAP - 1 - (q1 + __popcll(bb & below))] = e;
  };
  // evaluations of a front/back queue pair: the front entries one lane each
  // (weight-class), the back entries a quad each.  decode(e, l, i, j, bx, by)
  // gives an entry's window cell l, grid cell (i, j) and target pixel;
  // done(e, l, cost) is called once per entry, on the evaluating lane (the
  // quad's lane 0)
  [[maybe_unused]] auto run_queues = [&](int flen, int blen, auto decode, auto done) {
    for (int base = 0; base < flen; base += kThreads) {
      const int q = base + tid;
      bool own = false;
      if (q < flen) {
        const int e = s_queue[q];
        int l, i, j, bx, by;
        decode(e, l, i, j, bx, by);
        done(e, l, evalw(i, j, bx, by));
        own = owned(i, j);
      }
      count_work(q < flen, own);
    }
    for (int base = 0; base < blen; base += kQuads) {
      const int q = base + (tid >> 2);
      bool own = false;
      if (q < blen) {
        const int e = s_queue[QCAP - 1 - q];
        int l, i, j, bx, by;
        decode(e, l, i, j, bx, by);
        const uint32_t c = evalg(i, j, bx, by);
        if (qr == 0) done(e, l, c);
        own = owned(i, j);
      }
      count_work(q < blen && qr == 0, own);
    }
  };
  // queue append of the lanes with `on` set (one LDS atomic per wave)
  auto enqueue = [&](bool on, uint16_t e, unsigned int &len) {
    const uint64_t b = __ballot(on);
    int q0 = 0;
    if ((tid & 63) == 0 && b) q0 = (int)atomicAdd(&len, (unsigned)__popcll(b));
    q0 = __shfl(q0, 0);
    const int lane = tid & 63;
    if (on) s_queue[q0 + __popcll(b & (lane ? (~0ull >> (64 - lane)) : 0ull))] = e;
  };

  int ml = a.halo[0], mr = a.halo[1], mt = a.halo[2], mb = a.halo[3];
  // a random search follows step t unless t ends its group (the R^+ steps
  // of Flow Fields+ end at P - 1, the scale at T - 1)
  auto rs_after = [&](int t) { return t != a.P - 1 && t != a.T - 1; };
  // random-search candidate of cell (i, j) at step t from its current state
  // (branch-free, so that two draws in one block can interleave)
  [[maybe_unused]] auto rs_candidate = [&](int i, int j, int l, int t, int32_t &fc) {
    const uint32_t c0 = s_cost[l];
    const int32_t f0 = s_flow[l];
    int ox, oy;
    ffk::rs_offset(a.seed, d.stream_id, a.level, t, j, i, t < a.P ? a.Rnp : a.Rn, ox, oy);
    const int fx = ffk::flow_x(f0) + ox, fy = ffk::flow_y(f0) + oy;
    const int tx = i * n + fx, ty = j * n + fy;
    fc = ffk::pack_flow(fx, fy);
    return c0 != kUnset && (ox | oy) != 0 && tx >= 0 && tx < W && ty >= 0 && ty < H;
  };

  // initial state of the valid window: the state of every cell of a thread
  // is loaded first, then stored, evaluated (one lane per evaluation) or
  // queued (quads)
  {
    const int rl = max(ti0 - ml, 0), rr = min(oi1 + mr, Wn), rt = max(tj0 - mt, 0), rb = min(oj1 + mb, Hn);
    const int rw = rr - rl, rh = rb - rt;
    const int Wc = (Wn + 1) >> 1;
    constexpr int NI = (G::LH * G::LW + kThreads - 1) / kThreads;
    int32_t fv[NI];
    uint32_t cv[NI];
    bool ev[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = it * kThreads + tid;
      fv[it] = 0;
      cv[it] = kUnset;
      ev[it] = false;
      if (k < rw * rh) {
        const int i = rl + k % rw, j = rt + k / rw;
        if (a.mode == ffh::kLevelContinue) {
          fv[it] = d.flow_in[(size_t)j * Wn + i];
          cv[it] = d.cost_in[(size_t)j * Wn + i];
        } else if (a.mode == ffh::kLevelInit) {
          const uint32_t q = (uint32_t)d.nn_key[(size_t)j * Wn + i];
          fv[it] = ffk::pack_flow((int)(q % (uint32_t)W) - i * n, (int)(q / (uint32_t)W) - j * n);
          ev[it] = true;
        } else if (!((i | j) & 1)) {
          const int kc = (j >> 1) * Wc + (i >> 1);
          const uint32_t cc = d.ccost[kc];
          const int32_t cf = d.cflow[kc];
          if (cc != kUnset) {
            fv[it] = cf;
            ev[it] = true;
          }
        }
      }
    }
    // the staged descriptors go to LDS once both groups of loads are issued
    if constexpr (WF) {
#pragma unroll
      for (int it = 0; it < NS; ++it)
        if (it * kThreads + tid < NSTAGE) s_wa[it * kThreads + tid] = sv[it];
    } else if constexpr (!F32) {
      if constexpr (!SUB) {
#pragma unroll
        for (int it = 0; it < NS; ++it)
          if (it * kThreads + tid < G::DH * G::DW) s_da[it * kThreads + tid] = sv[it];
      }
    } else {
#pragma unroll
      for (int it = 0; it < NS; ++it)
        if (it * kThreads + tid < 4 * G::DH * G::DW) s_daf[it * kThreads + tid] = sf[it];
    }
    // one-lane seed evaluations read the staged descriptors, and queueing
    // needs the counters cleared: a barrier, except for a continuing run of
    // the quad kernels, which neither evaluates nor queues here
    if (!QUAD || a.mode != ffh::kLevelContinue) __syncthreads();
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = it * kThreads + tid;
      int cnt = 0, l = 0;
      bool inn = false;
      if (k < rw * rh) {
        const int i = rl + k % rw, j = rt + k / rw;
        l = (j - gj0) * G::LW + (i - gi0);
        s_flow[l] = fv[it];
        s_cost[l] = cv[it];
        if (ev[it]) {
          if constexpr (!QUAD) s_cost[l] = evalc(i, j, i * n + ffk::flow_x(fv[it]), j * n + ffk::flow_y(fv[it]));
          if constexpr (WF) inn = inner(i, j, i * n + ffk::flow_x(fv[it]), j * n + ffk::flow_y(fv[it]));
          cnt = owned(i, j);
        }
      }
      if constexpr (!QUAD) count_work(k < rw * rh && ev[it], cnt != 0);
      if constexpr (WF)
        enqueue2(k < rw * rh && ev[it], inn, (uint16_t)l, s_qlen, s_blen);
      else if constexpr (QUAD)
        enqueue(k < rw * rh && ev[it], (uint16_t)l, s_qlen);
      const int tot = __popcll(__ballot(cnt));
      if ((tid & 63) == 0 && tot) atomicAdd(&s_cnt, (unsigned)tot);
    }
  }
  __syncthreads();
  if constexpr (WF) {
    if (a.mode != ffh::kLevelContinue) {  // the seed evaluations
      run_queues(
          (int)s_qlen, (int)s_blen,
          [&](int e, int &l, int &i, int &j, int &bx, int &by) {
            l = e;
            i = gi0 + l % G::LW;
            j = gj0 + l / G::LW;
            const int32_t f = s_flow[l];
            bx = i * n + ffk::flow_x(f);
            by = j * n + ffk::flow_y(f);
          },
          [&](int, int l, uint32_t c) { s_cost[l] = c; });
      __syncthreads();
      if (tid == 0) s_qlen = s_blen = 0;
      __syncthreads();
    }
  } else if constexpr (QUAD) {
    if (a.mode != ffh::kLevelContinue) {  // the seed evaluations, a quad each
      const int qlen = (int)s_qlen;
      for (int base = 0; base < qlen; base += kQuads) {
        const int q = base + (tid >> 2);
        bool own = false;
        if (q < qlen) {
          const int l = s_queue[q], i = gi0 + l % G::LW, j = gj0 + l / G::LW;
          const int32_t f = s_flow[l];
          const uint32_t c = evalq(i, j, i * n + ffk::flow_x(f), j * n + ffk::flow_y(f));
          if (qr == 0) s_cost[l] = c;
          own = owned(i, j);
        }
        count_work(q < qlen && qr == 0, own);
      }
      __syncthreads();
      if (tid == 0) s_qlen = 0;
      __syncthreads();
    }
  }

  for (int t = a.t_begin; t < a.t_end; ++t) {
    const int dir = t & 3;
    const int hdi = (dir == 0 || dir == 3) ? -1 : 1;
    const int vdj = (dir == 0 || dir == 2) ? -1 : 1;
    for (int colour = 1; colour >= 0; --colour) {
      if (hdi < 0) --ml; else --mr;
      if (vdj < 0) --mt; else --mb;
      const int rl = max(ti0 - ml, 0), rr = min(oi1 + mr, Wn), rt = max(tj0 - mt, 0), rb = min(oj1 + mb, Hn);
      const int hw = (rr - rl + 1) >> 1, rh = rb - rt;
      // k / hw as a multiply-high by ceil(2^32 / hw): exact for k, hw < 2^16
      // (the error term k (m - 2^32 / hw) / 2^32 stays below 1 / hw)
      const uint32_t hwm = hw > 1 ? 0xFFFFFFFFu / (uint32_t)hw + 1u : 0u;
      // Cells of this colour in the valid window, thread-strided.
      auto cell_of = [&](int c, int k, int &i, int &j) {
        const int q = hw > 1 ? (int)__umulhi((uint32_t)k, hwm) : k;
        j = rt + (k < hw * rh ? q : 0);
        i = rl + ((c + j + rl) & 1) + 2 * (hw > 1 ? k - q * hw : 0);
        return k < hw * rh && i < rr;
      };
      auto cell = [&](int k, int &i, int &j) { return cell_of(colour, k, i, j); };
      // (1) candidate checks (Eq. 2 with the skip rules).  Only evaluations
      // whose value can matter are queued: the vertical source is not
      // evaluated when it repeats the horizontal one or the cell's own flow
      // (its value is then known not to win).  The cell's cost slot holds
      // the key cost*4 + rank (own 0, horizontal 1, vertical 2; UNSET stays
      // all ones) and evaluations lower it with an LDS atomic min: the
      // smallest key is exactly the sequential strict-< choice with ties
      // kept by the earlier candidate.
      for (int base = 0; base < hw * rh; base += kThreads) {
        int i, j;
        const bool live = cell(base + tid, i, j);
        const int l = (j - gj0) * G::LW + (i - gi0);
        bool hv = false, vcomp = false;
        [[maybe_unused]] bool hin = false, vin = false;  // weight-class path: cell and target inside
        if (live) {
          // the state of the cell and of both sources in one round of LDS
          // reads: a source cell lies inside the window for every live cell
          // (the valid region shrinks towards it), so the reads need no
          // guard; an outside-grid source's slot holds nothing used
          const int lh = l + hdi, lv = l + vdj * G::LW;
          uint32_t c0 = s_cost[l], chs = s_cost[lh], cvs = s_cost[lv];
          int32_t f0 = s_flow[l], fhs = s_flow[lh], fvs = s_flow[lv];
          // keeps the compiler from sinking the reads into the branches below
          asm volatile("" : "+v"(c0), "+v"(chs), "+v"(cvs), "+v"(f0), "+v"(fhs), "+v"(fvs));
          const bool set0 = c0 != kUnset;
          const int x = i * n, y = j * n;
          bool vb = false, vsame_h = false, vsame_0 = false;
          int32_t fh = 0;
          if (i + hdi >= 0 && i + hdi < Wn && chs != kUnset) {
            fh = fhs;
            const int tx = x + ffk::flow_x(fh), ty = y + ffk::flow_y(fh);
            hv = !(set0 && fh == f0) && tx >= 0 && tx < W && ty >= 0 && ty < H;
            if constexpr (WF) hin = inner(i, j, tx, ty);
          }
          if (j + vdj >= 0 && j + vdj < Hn && cvs != kUnset) {
            const int32_t fv = fvs;
            const int tx = x + ffk::flow_x(fv), ty = y + ffk::flow_y(fv);
            vb = tx >= 0 && tx < W && ty >= 0 && ty < H;
            vsame_h = hv && fv == fh;
            vsame_0 = set0 && fv == f0;
            if constexpr (WF) vin = inner(i, j, tx, ty);
          }
          vcomp = vb && !vsame_h && !vsame_0;
          s_flags[l] = (uint8_t)(hv | (vb << 1) | (vsame_h << 2) | (vsame_0 << 3) | (vcomp << 4));
          if constexpr (F32)
            s_key[l] = set0 ? (unsigned long long)c0 << 2 : ~0ull;
          else
            s_cost[l] = set0 ? c0 << 2 : kUnset;
        }
        if constexpr (WF) {  // weight-class entries at the front, descriptor quads at the back
          const uint64_t bhi = __ballot(hv && hin), bvi = __ballot(vcomp && vin);
          const uint64_t bhb = __ballot(hv && !hin), bvb = __ballot(vcomp && !vin);
          const int nhi = __popcll(bhi), nvi = __popcll(bvi), nhb = __popcll(bhb), nvb = __popcll(bvb);
          int q0 = 0, q1 = 0;
          if ((tid & 63) == 0) {
            if (nhi + nvi) q0 = (int)atomicAdd(&s_qlen, (unsigned)(nhi + nvi));
            if (nhb + nvb) q1 = (int)atomicAdd(&s_blen, (unsigned)(nhb + nvb));
          }
          q0 = __shfl(q0, 0);
          q1 = __shfl(q1, 0);
          const int lane = tid & 63;
          const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
          if (hv && hin) s_queue[q0 + __popcll(bhi & below)] = (uint16_t)(l << 1);
          if (vcomp && vin) s_queue[q0 + nhi + __popcll(bvi & below)] = (uint16_t)((l << 1) | 1);
          if (hv && !hin) s_queue[QCAP - 1 - (q1 + __popcll(bhb & below))] = (uint16_t)(l << 1);
          if (vcomp && !vin) s_queue[QCAP - 1 - (q1 + nhb + __popcll(bvb & below))] = (uint16_t)((l << 1) | 1);
        } else {
          const uint64_t bh = __ballot(hv), bv = __ballot(vcomp);
          const int nh = __popcll(bh), nv = __popcll(bv);
          int q0 = 0;
          if ((tid & 63) == 0 && nh + nv) q0 = (int)atomicAdd(&s_qlen, (unsigned)(nh + nv));
          q0 = __shfl(q0, 0);
          const int lane = tid & 63;
          const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
          if (hv) s_queue[q0 + __popcll(bh & below)] = (uint16_t)(l << 1);
          if (vcomp) s_queue[q0 + nh + __popcll(bv & below)] = (uint16_t)((l << 1) | 1);
        }
      }
      __syncthreads();
      // (2) the queued evaluations, densely over all lanes
      if constexpr (WF) {
        run_queues(
            (int)s_qlen, (int)s_blen,
            [&](int e, int &l, int &i, int &j, int &bx, int &by) {
              l = e >> 1;
              i = gi0 + l % G::LW;
              j = gj0 + l / G::LW;
              const int32_t f = s_flow[(e & 1) ? l + vdj * G::LW : l + hdi];
              bx = i * n + ffk::flow_x(f);
              by = j * n + ffk::flow_y(f);
            },
            [&](int e, int l, uint32_t c) { atomicMin(&s_cost[l], (c << 2) | (uint32_t)(1 + (e & 1))); });
      } else if constexpr (QUAD) {
        const int qlen = (int)s_qlen;
        for (int base = 0; base < qlen; base += kQuads) {
          const int q = base + (tid >> 2);
          bool own = false;
          if (q < qlen) {
            const int e = s_queue[q], l = e >> 1, vert = e & 1;
            const int i = gi0 + l % G::LW, j = gj0 + l / G::LW;
            const int32_t f = s_flow[vert ? l + vdj * G::LW : l + hdi];
            const uint32_t c = evalq(i, j, i * n + ffk::flow_x(f), j * n + ffk::flow_y(f));
            if (qr == 0) {
              if constexpr (F32)
                atomicMin(&s_key[l], ((unsigned long long)c << 2) | (unsigned long long)(1 + vert));
              else
                atomicMin(&s_cost[l], (c << 2) | (uint32_t)(1 + vert));
            }
            own = owned(i, j);
          }
          count_work(q < qlen && qr == 0, own);
        }
      } else {
        const int qlen = (int)s_qlen;
        for (int base = 0; base < qlen; base += kThreads) {
          const int q = base + tid;
          bool own = false;
          if (q < qlen) {
            const int e = s_queue[q], l = e >> 1, vert = e & 1;
            const int i = gi0 + l % G::LW, j = gj0 + l / G::LW;
            const int32_t f = s_flow[vert ? l + vdj * G::LW : l + hdi];
            const uint32_t c = evalc(i, j, i * n + ffk::flow_x(f), j * n + ffk::flow_y(f));
            atomicMin(&s_cost[l], (c << 2) | (uint32_t)(1 + vert));
            own = owned(i, j);
          }
          count_work(q < qlen, own);
        }
      }
      __syncthreads();
      if (tid == 0) s_qlen = s_blen = 0;
      // (3) new state and evaluation count of every cell
      for (int base = 0; base < hw * rh; base += kThreads) {
        int i, j;
        const bool live = cell(base + tid, i, j);
        const int l = (j - gj0) * G::LW + (i - gi0);
        int cnt = 0;
        if (live) {
          // both source flows read with the key and flags (one round of
          // LDS reads; the sources lie inside the window, as in the check)
          int32_t fhs = s_flow[l + hdi], fvs = s_flow[l + vdj * G::LW];
          asm volatile("" : "+v"(fhs), "+v"(fvs));
          bool unset;
          int rank;
          uint32_t cost;
          if constexpr (F32) {
            const unsigned long long key = s_key[l];
            unset = key == ~0ull;
            rank = unset ? 0 : (int)(key & 3);
            cost = unset ? kUnset : (uint32_t)(key >> 2);
          } else {
            const uint32_t key = s_cost[l];
            unset = key == kUnset;
            rank = unset ? 0 : (int)(key & 3);
            cost = unset ? kUnset : key >> 2;
          }
          const int fl = s_flags[l];
          const bool hv = fl & 1, vb = fl & 2, vsame_h = fl & 4, vsame_0 = fl & 8;
          cnt = hv;
          // the vertical source counts as evaluated unless it equals the
          // best flow after the horizontal step
          if (vb) cnt += vsame_h ? (rank == 0) : vsame_0 ? (rank == 1) : 1;
          if (rank) s_flow[l] = rank == 1 ? fhs : fvs;
          s_cost[l] = cost;
          if (!owned(i, j)) cnt = 0;
        }
        if constexpr (QUAD) {
          // after the second half-sweep of a step with a random search:
          // the cell is final, draw its candidate now, and that of the cell
          // of the other colour with the same index (final since the first
          // half-sweep; the same number of cells): the two hashes are
          // independent, so they run interleaved
          if (colour == 0 && rs_after(t)) {
            int i1, j1;
            const bool live1 = cell_of(1, base + tid, i1, j1);
            const int l1 = (j1 - gj0) * G::LW + (i1 - gi0);
            int32_t fc = 0, fc1 = 0;
            bool act = false, act1 = false;
            if (__ballot(live || live1)) {  // (a cell index past the valid region reads slot 0)
              act = rs_candidate(i, j, live ? l : 0, t, fc) && live;
              act1 = rs_candidate(i1, j1, live1 ? l1 : 0, t, fc1) && live1;
            }
            if (act) {
              s_flags[l] = (uint32_t)fc;
              cnt += owned(i, j);
            }
            if (act1) s_flags[l1] = (uint32_t)fc1;
            const int tot1 = __popcll(__ballot(act1 && owned(i1, j1)));
            if ((tid & 63) == 0 && tot1) atomicAdd(&s_cnt, (unsigned)tot1);
            if constexpr (WF) {
              enqueue2(act, act && inner(i, j, i * n + ffk::flow_x(fc), j * n + ffk::flow_y(fc)), (uint16_t)l, s_rlen,
                       s_rblen);
              enqueue2(act1, act1 && inner(i1, j1, i1 * n + ffk::flow_x(fc1), j1 * n + ffk::flow_y(fc1)),
                       (uint16_t)l1, s_rlen, s_rblen);
            } else {
              enqueue(act, (uint16_t)l, s_rlen);
              enqueue(act1, (uint16_t)l1, s_rlen);
            }
          }
        }
        const int tot = __popcll(__ballot(cnt >= 1)) + __popcll(__ballot(cnt >= 2)) + __popcll(__ballot(cnt >= 3));
        if ((tid & 63) == 0 && tot) atomicAdd(&s_cnt, (unsigned)tot);
      }
      __syncthreads();
    }
    if (WF && rs_after(t)) {  // the candidates drawn in the second half-sweep
      run_queues(
          (int)s_rlen, (int)s_rblen,
          [&](int e, int &l, int &i, int &j, int &bx, int &by) {
            l = e;
            i = gi0 + l % G::LW;
            j = gj0 + l / G::LW;
            const int32_t fc = (int32_t)s_flags[l];
            bx = i * n + ffk::flow_x(fc);
            by = j * n + ffk::flow_y(fc);
          },
          [&](int, int l, uint32_t c) {
            if (c < s_cost[l]) {
              s_cost[l] = c;
              s_flow[l] = (int32_t)s_flags[l];
            }
          });
      __syncthreads();
      if (tid == 0) s_rlen = s_rblen = 0;  // next written after the next step's first half-sweep
    } else if (QUAD && rs_after(t)) {  // the candidates drawn in the second half-sweep, a quad each
      const int qlen = (int)s_rlen;
      for (int base = 0; base < qlen; base += kQuads) {
        const int q = base + (tid >> 2);
        bool own = false;
        if (q < qlen) {
          const int l = s_queue[q], i = gi0 + l % G::LW, j = gj0 + l / G::LW;
          const int32_t fc = (int32_t)s_flags[l];
          const uint32_t e = evalq(i, j, i * n + ffk::flow_x(fc), j * n + ffk::flow_y(fc));
          if (qr == 0 && e < s_cost[l]) {
            s_cost[l] = e;
            s_flow[l] = fc;
          }
          own = owned(i, j);
        }
        count_work(q < qlen && qr == 0, own);
      }
      __syncthreads();
      if (tid == 0) s_rlen = 0;  // next written after the next step's first half-sweep
    } else if (rs_after(t)) {  // random search over the whole valid window
      const int rl = max(ti0 - ml, 0), rr = min(oi1 + mr, Wn), rt = max(tj0 - mt, 0), rb = min(oj1 + mb, Hn);
      const int rw = rr - rl, rh = rb - rt;
      for (int base = 0; base < rw * rh; base += kThreads) {
        const int k = base + tid;
        const bool live = k < rw * rh;
        const int i = rl + (live ? k % rw : 0), j = rt + (live ? k / rw : 0);
        const int l = (j - gj0) * G::LW + (i - gi0);
        bool act = false;
        int fx = 0, fy = 0;
        uint32_t c0 = kUnset;
        if (live) {
          c0 = s_cost[l];
          if (c0 != kUnset) {
            int ox, oy;
            ffk::rs_offset(a.seed, d.stream_id, a.level, t, j, i, t < a.P ? a.Rnp : a.Rn, ox, oy);
            const int32_t f0 = s_flow[l];
            fx = ffk::flow_x(f0) + ox;
            fy = ffk::flow_y(f0) + oy;
            const int tx = i * n + fx, ty = j * n + fy;
            act = (ox | oy) != 0 && tx >= 0 && tx < W && ty >= 0 && ty < H;
          }
        }
        int cnt = 0;
        if (act) {
          const uint32_t e = evalc(i, j, i * n + fx, j * n + fy);
          cnt = owned(i, j);
          if (e < c0) {
            s_cost[l] = e;
            s_flow[l] = ffk::pack_flow(fx, fy);
          }
        }
        count_work(act, cnt != 0);
        const int tot = __popcll(__ballot(cnt));
        if ((tid & 63) == 0 && tot) atomicAdd(&s_cnt, (unsigned)tot);
      }
      __syncthreads();
    }
  }

  // write back the owned tile
  const int ow = oi1 - ti0, oh = oj1 - tj0;
  for (int k = tid; k < ow * oh; k += kThreads) {
    const int i = ti0 + k % ow, j = tj0 + k / ow;
    const int l = (j - gj0) * G::LW + (i - gi0);
    d.flow[(size_t)j * Wn + i] = s_flow[l];
    d.cost[(size_t)j * Wn + i] = s_cost[l];
  }
  if (tid == 0 && s_cnt && d.n_evals) atomicAdd(d.n_evals, (unsigned long long)s_cnt);
  if (tid == 0 && d.n_work && s_work[1]) {
    atomicAdd(d.n_work, (unsigned long long)s_work[0]);
    atomicAdd(d.n_work + 1, (unsigned long long)s_work[1]);
  }
}

// Waves per SIMD a kernel is compiled for: four (two with EV = 2), so that
// the register budget keeps the loads of a patch in flight together instead
// of one after another; five for the weight-class kernels (EV = 4) whose LDS
// window lets five waves per SIMD be resident (their 13 row loads fit 80
// registers; measured 1.6 % faster per pair at 1024x436), and up to seven
// for the smaller weight-class tiles whose window lets six or seven
// workgroups share a compute unit: the launch is bound by the latency of
// its barrier-separated phases, which more resident workgroups hide.
template <int TW, int TH, int kThreads, int EV, int HALO>
constexpr int level_waves() {
  if constexpr (EV == 2) return 2;
  if constexpr (EV != 4) return 4;
  using G = Geo<TW, TH, HALO>;
  constexpr int lds = G::LH * G::LW * 14 + (G::LH + 12) * G::LW * 16;  // state, flags, queue; image a's rows
  constexpr int fit = 160 * 1024 / lds * (kThreads / 64) / 4;           // waves per SIMD the LDS allows
  // a tile whose area is not a power of two (32x12) is sized for six or
  // seven resident workgroups
  if constexpr (kThreads == 256 && ((TW * TH) & (TW * TH - 1)) != 0) return fit < 5 ? 4 : (fit > 7 ? 7 : fit);
  return fit >= 5 ? 5 : 4;
}

// One workgroup per (direction, tile) of one pair; XCD-aware order.
template <int LOG2N, int TW, int TH, int kThreads, int EV, int HALO, int RR = kR>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    EV >= 3 ? level_waves<TW, TH, kThreads, EV, HALO>() : 1, level_waves<TW, TH, kThreads, EV, HALO>()))) void k_level(ffh::LevelKArgs a) {
  const int tiles = a.tiles_x * ((a.Hn + TH - 1) / TH);
  const int wg = ffk::xcd_remap(blockIdx.x, gridDim.x);
  level_body<LOG2N, TW, TH, kThreads, EV, false, HALO, RR>(a, a.dir[wg / tiles], wg % tiles);
}

// A sub-scale stage (Sec. 3.3: patch scale a.sub_m on the grid of scale n):
// the radius-3 descriptor-quad kernel reading both images' image-order maps.
template <int LOG2N, int TW, int TH, int kThreads, int HALO>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    level_waves<TW, TH, kThreads, 3, HALO>(), level_waves<TW, TH, kThreads, 3, HALO>()))) void k_level_sub(ffh::LevelKArgs a) {
  const int tiles = a.tiles_x * ((a.Hn + TH - 1) / TH);
  const int wg = ffk::xcd_remap(blockIdx.x, gridDim.x);
  level_body<LOG2N, TW, TH, kThreads, 3, false, HALO, kR, true>(a, a.dir[wg / tiles], wg % tiles);
}

// Float learned features (padded float maps in LevelKDir::Da/Db).
template <int LOG2N, int TW, int TH, int kThreads, int HALO>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 3))) void k_level_f32(
    ffh::LevelKArgs a) {
  const int tiles = a.tiles_x * ((a.Hn + TH - 1) / TH);
  const int wg = ffk::xcd_remap(blockIdx.x, gridDim.x);
  level_body<LOG2N, TW, TH, kThreads, 1, true, HALO>(a, a.dir[wg / tiles], wg % tiles);
}

// Persistent launch over the (pair, direction, tile) items of a batch.
template <int LOG2N, int TW, int TH, int kThreads, int EV, int HALO>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    EV >= 3 ? level_waves<TW, TH, kThreads, EV, HALO>() : 1, level_waves<TW, TH, kThreads, EV, HALO>()))) void k_level_batch(
    ffh::LevelKArgs base, ffh::BatchStage st) {
  constexpr int n = 1 << LOG2N;
  ffk::for_items(st.total, [&](int item) {
    const int p = ffk::batch_pair(st.prefix, st.npairs, item);
    const ffh::BatchPair &bp = st.pairs[p];
    ffh::LevelKArgs a = base;
    a.W = bp.W;
    a.H = bp.H;
    a.Wn = (bp.W + n - 1) / n;
    a.Hn = (bp.H + n - 1) / n;
    a.tiles_x = (a.Wn + TW - 1) / TW;
    const int tiles = a.tiles_x * ((a.Hn + TH - 1) / TH);
    const int local = item - st.prefix[p];
    const int dir = local / tiles, lv = st.lv;
    ffh::LevelKDir d;
    d.Da = bp.desc[dir][lv];
    d.Db = bp.desc[dir ^ 1][lv];
    d.Wa = bp.wform[dir][lv];
    d.Wb = bp.wform[dir ^ 1][lv];
    d.flow = st.dst ? bp.sflow[lv][dir] : bp.gflow[lv][dir];
    d.cost = st.dst ? bp.scost[lv][dir] : bp.gcost[lv][dir];
    d.flow_in = st.src ? bp.sflow[lv][dir] : bp.gflow[lv][dir];
    d.cost_in = st.src ? bp.scost[lv][dir] : bp.gcost[lv][dir];
    d.cflow = lv + 1 < st.L ? bp.gflow[lv + 1][dir] : nullptr;
    d.ccost = lv + 1 < st.L ? bp.gcost[lv + 1][dir] : nullptr;
    d.nn_key = bp.keys[dir];
    d.n_evals = bp.evals + dir;
    d.n_work = nullptr;
    d.stream_id = dir;
    level_body<LOG2N, TW, TH, kThreads, EV, false, HALO>(a, d, local % tiles);
    __syncthreads();  // the next item reuses the LDS window
  });
}

template <int LOG2N, int TW, int TH, int THREADS, int EV, int HALO = ffh::kLevelHalo, int RR = kR>
hipError_t launch_v(const ffh::LevelKArgs &a, const ffh::BatchStage *batch, hipStream_t stream) {
  if constexpr (RR != kR) {
    if (batch) return hipErrorInvalidValue;  // batches run radius 3
  } else if (batch) {
    if (batch->total <= 0) return hipSuccess;
    // persistent: enough workgroups to fill the chip, a multiple of 8
    const int grid = ((std::min(batch->total, 2048) + 7) / 8) * 8;
    hipLaunchKernelGGL((k_level_batch<LOG2N, TW, TH, THREADS, EV, HALO>), dim3(grid), dim3(THREADS), 0, stream, a,
                       *batch);
    return hipGetLastError();
  }
  ffh::LevelKArgs b = a;
  b.tiles_x = (a.Wn + TW - 1) / TW;
  const int tiles = b.tiles_x * ((a.Hn + TH - 1) / TH);
  if (a.sub_m) {
    if constexpr (EV == 3 && RR == kR) {
      hipLaunchKernelGGL((k_level_sub<LOG2N, TW, TH, THREADS, HALO>), dim3(tiles * a.ndir), dim3(THREADS), 0, stream,
                         b);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  hipLaunchKernelGGL((k_level<LOG2N, TW, TH, THREADS, EV, HALO, RR>), dim3(tiles * a.ndir), dim3(THREADS), 0, stream,
                     b);
  return hipGetLastError();
}

template <int LOG2N, int TW, int TH, int THREADS, int HALO>
hipError_t launch_f32(const ffh::LevelKArgs &a, hipStream_t stream) {
  ffh::LevelKArgs b = a;
  b.tiles_x = (a.Wn + TW - 1) / TW;
  const int tiles = b.tiles_x * ((a.Hn + TH - 1) / TH);
  hipLaunchKernelGGL((k_level_f32<LOG2N, TW, TH, THREADS, HALO>), dim3(tiles * a.ndir), dim3(THREADS), 0, stream,
                     b);
  return hipGetLastError();
}

// Float-feature variant index -> kernel; kHaloF32 in ff_level.hip lists the
// window halo of every index, which must match.  16x16 or 8x8 tiles (the
// latter for the small grids of the coarse scales); a halo of 2 allows one
// step per launch, 4 two and 6 three.
template <int LOG2N>
hipError_t launch_nf32(const ffh::LevelKArgs &a, int variant, hipStream_t stream) {
  switch (variant) {
    case 0: return launch_f32<LOG2N, 16, 16, 256, 2>(a, stream);
    case 1: return launch_f32<LOG2N, 8, 8, 256, 2>(a, stream);
    case 2: return launch_f32<LOG2N, 8, 8, 256, 4>(a, stream);
    case 3: return launch_f32<LOG2N, 8, 8, 256, 6>(a, stream);
    case 4: return launch_f32<LOG2N, 16, 16, 256, 4>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

// Variant index -> kernel; the tile and halo of every index are listed in
// kVariants (ff_level.hip), which must match.
template <int LOG2N>
hipError_t launch_n(const ffh::LevelKArgs &a, const ffh::BatchStage *batch, int variant, hipStream_t stream) {
  switch (variant) {
    case 0: return launch_v<LOG2N, 64, 32, 1024, 0>(a, batch, stream);
    case 1: return launch_v<LOG2N, 32, 16, 1024, 0>(a, batch, stream);
    case 2: return launch_v<LOG2N, 32, 16, 256, 1>(a, batch, stream);
    case 3: return launch_v<LOG2N, 16, 16, 256, 1>(a, batch, stream);
    case 4: return launch_v<LOG2N, 32, 32, 512, 1>(a, batch, stream);
    case 5: return launch_v<LOG2N, 32, 16, 256, 2>(a, batch, stream);
    case 6: return launch_v<LOG2N, 16, 16, 256, 2>(a, batch, stream);
    case 7: return launch_v<LOG2N, 32, 32, 512, 2>(a, batch, stream);
    case 8: return launch_v<LOG2N, 8, 8, 256, 2>(a, batch, stream);
    case 9: return launch_v<LOG2N, 16, 16, 512, 2>(a, batch, stream);
    case 10: return launch_v<LOG2N, 16, 16, 1024, 1>(a, batch, stream);
    case 11: return launch_v<LOG2N, 16, 16, 256, 3, 2>(a, batch, stream);
    case 12: return launch_v<LOG2N, 32, 16, 256, 3, 2>(a, batch, stream);
    case 13: return launch_v<LOG2N, 16, 16, 256, 3>(a, batch, stream);
    case 14: return launch_v<LOG2N, 8, 8, 256, 3>(a, batch, stream);
    case 15: return launch_v<LOG2N, 8, 8, 256, 3, 2>(a, batch, stream);
    case 16: return launch_v<LOG2N, 32, 16, 256, 3, 4>(a, batch, stream);
    case 17: return launch_v<LOG2N, 16, 16, 256, 3, 4>(a, batch, stream);
    case 18: return launch_v<LOG2N, 32, 16, 256, 4, 4>(a, batch, stream);
    case 19: return launch_v<LOG2N, 16, 16, 256, 4, 4>(a, batch, stream);
    case 20: return launch_v<LOG2N, 32, 16, 256, 4, 2>(a, batch, stream);
    case 21: return launch_v<LOG2N, 16, 16, 256, 4, 2>(a, batch, stream);
    case 22: return launch_v<LOG2N, 8, 8, 256, 4, 6>(a, batch, stream);
    case 23: return launch_v<LOG2N, 8, 8, 256, 4, 2>(a, batch, stream);
    case 24: return launch_v<LOG2N, 32, 16, 512, 4, 4>(a, batch, stream);
    case 25: return launch_v<LOG2N, 64, 32, 1024, 4, 4>(a, batch, stream);
    case 26: return launch_v<LOG2N, 8, 8, 1024, 3>(a, batch, stream);
    case 27: return launch_v<LOG2N, 8, 8, 1024, 3, 4>(a, batch, stream);
    case 28: return launch_v<LOG2N, 8, 8, 1024, 4>(a, batch, stream);
    case 29: return launch_v<LOG2N, 8, 8, 1024, 4, 4>(a, batch, stream);
    case 30: return launch_v<LOG2N, 16, 16, 1024, 3>(a, batch, stream);
    case 31: return launch_v<LOG2N, 32, 12, 256, 4, 2>(a, batch, stream);
    case 32: return launch_v<LOG2N, 4, 4, 1024, 3, 4>(a, batch, stream);
    default: return hipErrorInvalidValue;
  }
}

// Patch radii 2 and 4 (the second backward field of Sec. 3.7 in the
// conference setting, r2 = 2; the radius r = 4 of Flow Fields+, Sec. 4.1):
// the descriptor-quad variants, same tiles and halos as the indices of
// launch_n; quad_variant in ff_level.hip maps every other index onto one of
// these with the same window halo.
template <int LOG2N, int RR>
hipError_t launch_n_rx(const ffh::LevelKArgs &a, int variant, hipStream_t stream) {
  switch (variant) {
    case 11: return launch_v<LOG2N, 16, 16, 256, 3, 2, RR>(a, nullptr, stream);
    case 12: return launch_v<LOG2N, 32, 16, 256, 3, 2, RR>(a, nullptr, stream);
    case 13: return launch_v<LOG2N, 16, 16, 256, 3, ffh::kLevelHalo, RR>(a, nullptr, stream);
    case 14: return launch_v<LOG2N, 8, 8, 256, 3, ffh::kLevelHalo, RR>(a, nullptr, stream);
    case 15: return launch_v<LOG2N, 8, 8, 256, 3, 2, RR>(a, nullptr, stream);
    case 16: return launch_v<LOG2N, 32, 16, 256, 3, 4, RR>(a, nullptr, stream);
    case 17: return launch_v<LOG2N, 16, 16, 256, 3, 4, RR>(a, nullptr, stream);
    case 26: return launch_v<LOG2N, 8, 8, 1024, 3, ffh::kLevelHalo, RR>(a, nullptr, stream);
    case 27: return launch_v<LOG2N, 8, 8, 1024, 3, 4, RR>(a, nullptr, stream);
    case 30: return launch_v<LOG2N, 16, 16, 1024, 3, ffh::kLevelHalo, RR>(a, nullptr, stream);
    default: return hipErrorInvalidValue;
  }
}


}  // namespace
