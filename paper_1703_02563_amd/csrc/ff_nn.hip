// Exact brute-force nearest neighbour of the coarsest-grid cells (stands in
// for the kd-tree candidate search of Sec. 3.1 with one candidate; the
// initial flow of Eq. 1 / Eq. 4 is F = q - p).
//
// ||a - b||^2 = |a|^2 + |b|^2 - 2 a.b is a dense contraction over the 16
// descriptor bytes.  Bytes v are shifted to int8 (v - 128, a plain xor with
// 0x80), which leaves the distance unchanged, and the dot products of 32
// queries x 32 references run on v_mfma_i32_32x32x16_i8 (exact in int32).
//
// Argmin with ties to the smallest reference index, without a compare and
// select per pair: per (query, reference) the lane forms the score
//     s = 4096 * dot - (2048 * |b|^2 + t) = -(2048 * (|b|^2 - 2 dot) + t)
// with t the tile index inside the current chunk (t < 2048), one
// v_lshl_add per pair, and keeps max(s) with v_max3 over two tiles.  Since
// |b|^2 - 2 dot = dist - |a|^2 lies in [-2^18, 2^20), s never overflows and
// max(s) is the smallest distance, then the smallest tile.  Within a lane
// the reference column is fixed, so (distance, tile) orders references by
// index.  At the end of the chunk each lane decodes its best, the 32 lanes
// holding the same queries reduce (distance, index) as one 64-bit key, and
// one atomicMin per query merges chunks and waves.
//
// Key written to global memory: ((dist - |a|^2 + 2^20) << 32) | index; the
// init kernel adds |a|^2 back.  Padding references (index >= N) carry
// |b|^2 = 2^20 - 1 and zero bytes, so their score is below every real one.
#include <algorithm>
#include <climits>

#include "ff_device.h"
#include "ff_internal.h"

namespace {

typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kTilesPerChunk = 512;   // batches; <= kMaxChunkTiles
constexpr int kMaxChunkTiles = 2048;  // the tile index inside a chunk must fit 11 bits
constexpr int kQB = 2;                // 32-query blocks per wave (B operand reuse)
constexpr int kWaves = 4;
constexpr int kNbPad = (1 << 20) - 1;

// Also clears the direction's NN keys (M <= N cells) for k_nn's atomicMin.
__global__ __launch_bounds__(256) void k_nn_norms(ffh::NNArgs a) {
  const ffh::NNDir d = a.dir[blockIdx.y];
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int Npad = (a.N + 31) & ~31;
  if (idx < a.M) d.keys[idx] = ~0ull;
  if (idx >= Npad) return;
  int s = kNbPad;
  if (idx < a.N) {
    const uint4 v = reinterpret_cast<const uint4 *>(d.Dr)[idx];
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
    s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int e = (int)((w[k] >> (8 * b)) & 0xFF) - 128;
        s += e * e;
      }
  }
  d.nb[idx] = s;
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t *dst, uint64_t value, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = value;
}

// Negation the compiler cannot see through: with an opaque addend,
// (acc << 12) + nk stays one v_lshl_add_u32 instead of a shift and a
// subtract.  Only the addend goes through asm; the matrix-core results are
// read by ordinary instructions, so the compiler keeps its MFMA
// read-after-write wait states.
__device__ __forceinline__ int opaque_neg(int v) {
  int r;
  asm("v_sub_u32 %0, 0, %1" : "=v"(r) : "v"(v));
  return r;
}

// Pins a loaded value to a register after `after` is computed (an empty
// asm with register operands; it touches no memory), so the load that
// produces it is waited for only at the end of the iteration that
// prefetches it.
__device__ __forceinline__ int pin(int v, int after) {
  asm volatile("" : "+v"(v) : "v"(after));
  return v;
}

__device__ __forceinline__ long load_i8x8(const uint8_t *p) {
  // 8 descriptor bytes -> 8 int8 (v - 128)
  return (long)(*reinterpret_cast<const unsigned long long *>(p) ^ 0x8080808080808080ull);
}

// Query block `qblk` (32 * kQB queries) against reference chunk `chunk` of
// one direction.  All threads of the workgroup call it.  kExcl: the next
// nearest reference instead of the nearest -- every reference whose key
// (distance, index) is at most the query's key in prev (the previous
// pass's result) is left out; prev[m] = ~0 leaves out all.
template <bool kExcl = false>
__device__ __forceinline__ void nn_body(const ffh::NNDir &d, int M, int N, int W, int nc, int Wc, int qblk,
                                        int chunk, int chunk_tiles, const uint64_t *prev = nullptr) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, kh = lane >> 5;
  const int ntiles = (N + 31) >> 5;
  const int m0 = qblk * (32 * kQB);
  const int t0 = chunk * chunk_tiles;
  const int t1 = min(t0 + chunk_tiles, ntiles);
  if (t0 + wave >= t1) return;  // wave-uniform: no tile for this wave
  struct {
    int Wc, nc;
  } a = {Wc, nc};

  long aop[kQB];
#pragma unroll
  for (int qb = 0; qb < kQB; ++qb) {
    const int m = min(m0 + qb * 32 + col, M - 1);
    const int i = m % a.Wc, j = m / a.Wc;
    const size_t pix = (size_t)(j * a.nc) * W + (size_t)(i * a.nc);
    aop[qb] = load_i8x8(d.Dq + pix * 16 + kh * 8);
  }

  int best[kQB][16];
#pragma unroll
  for (int qb = 0; qb < kQB; ++qb)
#pragma unroll
    for (int r = 0; r < 16; ++r) best[qb][r] = INT_MIN;
  // Exclusion as a score bound per (query row, lane): a reference of this
  // lane (column col, chunk tile tl, index (t0 + tl) * 32 + col) has a key
  // at most (dd*, q*) iff 2048 dd + tl <= K = 2048 dd* + floor((q* - col) /
  // 32) - t0 (the tile term clamped to [-1, 2047]), i.e. iff its score
  // -(2048 dd + tl) >= -K; it is kept iff the score is below thr = -K.
  int thr[kQB][16];
  if constexpr (kExcl) {
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + qb * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        int t = INT_MAX;  // padding rows: nothing left out (they write nothing)
        if (m < M) {
          const uint64_t pk = prev[m];
          if (pk == ~0ull) {
            t = INT_MIN;  // nothing left to find
          } else {
            const int dd = (int)(uint32_t)(pk >> 32) - (1 << 20);
            int tl = ((int)(uint32_t)pk - col) >> 5;  // floor: the shift is arithmetic
            tl = tl - t0 < -1 ? -1 : (tl - t0 > 2047 ? 2047 : tl - t0);
            t = (int)-(2048ll * dd + tl);  // 2048 dd + tl <= 2^31 - 1
          }
        }
        thr[qb][r] = t;
      }
  }

  const v16i zero = {0};
  // Operands of the two tiles of step t (the second repeats the first at the
  // odd tail).  The tile index is wave-uniform (scalar registers) and rides
  // in the buffer loads' scalar offset; references at or beyond N lie outside
  // the descriptor buffer's range (the loads return zeros, kept as zero
  // int8 bytes), and their padded norm keeps them below every real one.
  const __amdgpu_buffer_rsrc_t rdesc =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t *>(d.Dr), (short)0, N * 16, 0x00020000);
  const __amdgpu_buffer_rsrc_t rnorm =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t *>(d.nb), (short)0, ((N + 31) & ~31) * 4, 0x00020000);
  const int voff_desc = col * 16 + kh * 8, voff_norm = col * 4;
  struct Step {
    long ba, bb;
    int na, nb;
  };
  constexpr long kFlip = (long)0x8080808080808080ull;  // bytes v -> int8 v - 128
  auto fetch = [&](int t, int tb) {
    Step st;
    st.ba = (long)__builtin_amdgcn_raw_buffer_load_b64(rdesc, voff_desc, t * 512, 0) ^ (t * 32 + col < N ? kFlip : 0);
    st.bb = (long)__builtin_amdgcn_raw_buffer_load_b64(rdesc, voff_desc, tb * 512, 0) ^ (tb * 32 + col < N ? kFlip : 0);
    st.na = (int)__builtin_amdgcn_raw_buffer_load_b32(rnorm, voff_norm, t * 128, 0);
    st.nb = (int)__builtin_amdgcn_raw_buffer_load_b32(rnorm, voff_norm, tb * 128, 0);
    return st;
  };
  const int tw0 = t0 + __builtin_amdgcn_readfirstlane(wave);
  auto second = [&](int t) { return (t + kWaves < t1) ? t + kWaves : t; };
  Step cur = fetch(tw0, second(tw0));
  for (int t = tw0; t < t1; t += 2 * kWaves) {
    // the next step's operands are in flight while this step computes
    const int tn = t + 2 * kWaves < t1 ? t + 2 * kWaves : t;
    const Step nxt = fetch(tn, second(tn));
    const int tb = second(t);
    const long ba = cur.ba, bb = cur.bb;
    const int nka = opaque_neg((cur.na << 11) | (t - t0));
    const int nkb = opaque_neg((cur.nb << 11) | (tb - t0));
    // all four products first: the second pair runs on the matrix core
    // while the first pair's scores are reduced
    v16i acc_a[kQB], acc_b[kQB];
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
      acc_a[qb] = __builtin_amdgcn_mfma_i32_32x32x16_i8(aop[qb], ba, zero, 0, 0, 0);
      acc_b[qb] = __builtin_amdgcn_mfma_i32_32x32x16_i8(aop[qb], bb, zero, 0, 0, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int qb = 0; qb < kQB; ++qb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        int sa = acc_a[qb][r] * 4096 + nka;
        int sb = acc_b[qb][r] * 4096 + nkb;
        if constexpr (kExcl) {
          sa = sa < thr[qb][r] ? sa : INT_MIN;
          sb = sb < thr[qb][r] ? sb : INT_MIN;
        }
        best[qb][r] = max(best[qb][r], max(sa, sb));
      }
    }
    cur = nxt;
    cur.na = pin(cur.na, best[kQB - 1][15]);
    cur.nb = pin(cur.nb, best[kQB - 1][15]);
  }

#pragma unroll
  for (int qb = 0; qb < kQB; ++qb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int key = -best[qb][r];
      const int dd = key >> 11;        // dist - |a|^2
      const int tl = key & 2047;       // tile inside the chunk
      const uint32_t ref = (uint32_t)((t0 + tl) * 32 + col);
      unsigned long long v = ((unsigned long long)(uint32_t)(dd + (1 << 20)) << 32) | ref;
      if constexpr (kExcl) {
        if (best[qb][r] == INT_MIN) v = ~0ull;  // every reference of the lane left out
      }
#pragma unroll
      for (int off = 16; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off);
        v = o < v ? o : v;
      }
      const int row = 8 * (r >> 2) + 4 * kh + (r & 3);
      const int m = m0 + qb * 32 + row;
      if (col == 0 && m < M) atomicMin(reinterpret_cast<unsigned long long *>(d.keys) + m, v);
    }
}

__host__ __device__ __forceinline__ int nn_qblocks(int M) { return (M + 32 * kQB - 1) / (32 * kQB); }
__host__ __device__ __forceinline__ int nn_chunks(int N, int chunk_tiles = kTilesPerChunk) {
  return (((N + 31) >> 5) + chunk_tiles - 1) / chunk_tiles;
}

// One workgroup per (direction, reference chunk, query block) of one pair,
// query block fastest; XCD-aware order keeps the workgroups of one chunk on
// one L2.
__global__ __launch_bounds__(256) void k_nn(ffh::NNArgs a) {
  const int nqb = nn_qblocks(a.M), nchunk = nn_chunks(a.N, a.chunk_tiles);
  const int wg = ffk::xcd_remap(blockIdx.x, gridDim.x);
  nn_body(a.dir[wg / (nqb * nchunk)], a.M, a.N, a.W, a.nc, a.Wc, wg % nqb, (wg / nqb) % nchunk, a.chunk_tiles);
}

// ---- batches -----------------------------------------------------------
// Squared norms of both images' level-1 descriptors (items: pair, image,
// 256 references); the first item of a pair also clears its counters.
__global__ __launch_bounds__(256) void k_nn_norms_batch(ffh::BatchStage st) {
  ffk::for_items(st.total, [&](int item) {
    const int p = ffk::batch_pair(st.prefix, st.npairs, item);
    const ffh::BatchPair &bp = st.pairs[p];
    const int N = bp.W * bp.H, Npad = (N + 31) & ~31;
    const int blocks = (Npad + 255) / 256;
    const int local = item - st.prefix[p];
    const int im = local / blocks, idx = (local % blocks) * 256 + threadIdx.x;
    if (local == 0 && threadIdx.x < 2) bp.evals[threadIdx.x] = 0;
    if (idx >= Npad) return;
    int s = kNbPad;
    if (idx < N) {
      const uint4 v = reinterpret_cast<const uint4 *>(bp.desc1[im])[idx];
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
      s = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int e = (int)((w[k] >> (8 * b)) & 0xFF) - 128;
          s += e * e;
        }
    }
    bp.nb[im][idx] = s;
  });
}

// Key initialisation (items: pair, direction, 256 queries).
__global__ __launch_bounds__(256) void k_nn_fill_batch(ffh::BatchStage st) {
  ffk::for_items(st.total, [&](int item) {
    const int p = ffk::batch_pair(st.prefix, st.npairs, item);
    const ffh::BatchPair &bp = st.pairs[p];
    const int M = ((bp.W + st.n - 1) / st.n) * ((bp.H + st.n - 1) / st.n);
    const int blocks = (M + 255) / 256;
    const int local = item - st.prefix[p];
    const int dir = local / blocks, m = (local % blocks) * 256 + threadIdx.x;
    if (m < M) bp.keys[dir][m] = ~0ull;
  });
}

// NN of every pair (items: pair, direction, chunk, query block).
__global__ __launch_bounds__(256) void k_nn_batch(ffh::BatchStage st) {
  ffk::for_items(st.total, [&](int item) {
    const int p = ffk::batch_pair(st.prefix, st.npairs, item);
    const ffh::BatchPair &bp = st.pairs[p];
    const int nc = st.n, Wc = (bp.W + nc - 1) / nc;
    const int M = Wc * ((bp.H + nc - 1) / nc), N = bp.W * bp.H;
    const int nqb = nn_qblocks(M), nchunk = nn_chunks(N);
    const int local = item - st.prefix[p];
    const int dir = local / (nqb * nchunk);
    const ffh::NNDir d = {bp.desc1[dir], bp.desc1[dir ^ 1], bp.nb[dir ^ 1], bp.keys[dir]};
    nn_body(d, M, N, bp.W, nc, Wc, local % nqb, (local / nqb) % nchunk, kTilesPerChunk);
  });
}


// ---- the l nearest references (seed rerank, Eq. 1 / Eq. 4) -------------
//
// The k-th nearest reference of a query (k = 1 .. l - 1; k = 0 is k_nn's
// result) is the nearest one among those whose key (distance, index) is
// larger than the (k-1)-th's: pass k is k_nn with that exclusion, so l
// passes give the l smallest keys, ranked, with the ties of k_nn.

__global__ __launch_bounds__(256) void k_nn_excl(ffh::NNArgs a, ffh::TopLPrev prev) {
  const int nqb = nn_qblocks(a.M), nchunk = nn_chunks(a.N, a.chunk_tiles);
  const int wg = ffk::xcd_remap(blockIdx.x, gridDim.x);
  const int dir = wg / (nqb * nchunk);
  nn_body<true>(a.dir[dir], a.M, a.N, a.W, a.nc, a.Wc, wg % nqb, (wg / nqb) % nchunk, a.chunk_tiles,
                prev.key[dir]);
}

__device__ __forceinline__ int query_norm(const uint8_t *Dq, int W, int nc, int Wc, int m) {
  const int i = m % Wc, j = m / Wc;
  const uint4 v = reinterpret_cast<const uint4 *>(Dq)[(size_t)(j * nc) * W + (size_t)(i * nc)];
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  int s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int e = (int)((w[k] >> (8 * b)) & 0xFF) - 128;
      s += e * e;
    }
  return s;
}

// Reference index of the even-pixel subset (Flow Fields+ Fast x2: pixel
// (2a, 2b) is entry b * W2 + a) -> pixel index of the image.
__device__ __forceinline__ uint32_t even_pixel(uint32_t q, int W2, int W) {
  return (q / (uint32_t)W2) * 2u * (uint32_t)W + (q % (uint32_t)W2) * 2u;
}

// Level-1 descriptors of the pixels with even x and y, row-major [H2][W2].
__global__ __launch_bounds__(256) void k_gather_even(const uint4 *src, uint4 *dst, int W, int H) {
  const int W2 = (W + 1) >> 1, H2 = (H + 1) >> 1;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= W2 * H2) return;
  dst[k] = src[(size_t)(k / W2) * 2 * W + (k % W2) * 2];
}

// NN keys over the even-pixel subset -> keys naming image pixels.
__global__ __launch_bounds__(256) void k_remap_even(uint64_t *keys, int M, int W) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const uint64_t k = keys[m];
  if (k != ~0ull) keys[m] = (k & 0xFFFFFFFF00000000ull) | even_pixel((uint32_t)k, (W + 1) >> 1, W);
}

// Ranked candidates with the squared distance itself: cand[m * l + k] =
// (dist << 32) | q of pass k, ~0 for a pass that found no reference of the
// image (padding references, index >= N, or none left).
__global__ __launch_bounds__(256) void k_topl_assemble(ffh::TopLArgs a) {
  const ffh::TopLDir d = a.dir[blockIdx.y];
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= a.M) return;
  const int na = query_norm(d.Dq, a.W, a.nc, a.Wc, m);
  for (int k = 0; k < a.l; ++k) {
    const uint64_t rel = k == 0 ? d.nn_key[m] : d.keys[(size_t)(k - 1) * a.M + m];
    uint64_t out = ~0ull;
    if (rel != ~0ull && (int64_t)(uint32_t)rel < (int64_t)a.N) {
      const uint32_t q = a.even_refs ? even_pixel((uint32_t)rel, (a.W + 1) >> 1, a.W) : (uint32_t)rel;
      out = ((uint64_t)(uint32_t)((int)(uint32_t)(rel >> 32) - (1 << 20) + na) << 32) | q;
    }
    d.cand[(size_t)m * a.l + k] = out;
  }
}

}  // namespace

namespace ffh {

int batch_nn_items(int W, int H, int L) {
  const int nc = 1 << (L - 1);
  const int M = ((W + nc - 1) / nc) * ((H + nc - 1) / nc), N = W * H;
  const int nqb = (M + 32 * kQB - 1) / (32 * kQB);
  return 2 * nqb * nn_chunks(N);
}

static int persistent_grid(int total, int cap) { return ((std::min(std::max(total, 1), cap) + 7) / 8) * 8; }

hipError_t launch_batch_nn(const BatchStage &norms, const BatchStage &fill, const BatchStage &nn,
                           hipStream_t stream) {
  hipLaunchKernelGGL(k_nn_norms_batch, dim3(persistent_grid(norms.total, 4096)), dim3(256), 0, stream, norms);
  hipLaunchKernelGGL(k_nn_fill_batch, dim3(persistent_grid(fill.total, 4096)), dim3(256), 0, stream, fill);
  hipLaunchKernelGGL(k_nn_batch, dim3(persistent_grid(nn.total, 2048)), dim3(64 * kWaves), 0, stream, nn);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *dst, uint64_t value, int64_t count, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, dst, value, count);
  return hipGetLastError();
}

// Workgroups of k_nn the current device holds at once (compute units x
// resident workgroups per unit), cached per device.
static int nn_resident_workgroups() {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cache[dev] == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_nn, 64 * kWaves, 0) != hipSuccess)
      return 0;
    cache[dev] = std::max(cus * per_cu, 1);
  }
  return cache[dev];
}

// Reference chunk length: the number of chunks whose workgroups fill the
// device in the fewest rounds for the least work per workgroup (a grid of
// 1.2 rounds would leave most of the second round idle).  Each chunk also
// costs its reduction and merge, about as much as kChunkOverhead tiles.
static int nn_chunk_tiles(int ntiles, int per_chunk_wgs) {
  constexpr int kChunkOverhead = 64;
  const int cap = nn_resident_workgroups();
  const int min_chunks = (ntiles + kMaxChunkTiles - 1) / kMaxChunkTiles;
  if (cap <= 0) return std::max((ntiles + min_chunks - 1) / min_chunks, 1);
  // at least 32 tiles per chunk (8 per wave), at most 8 rounds' worth
  const int max_chunks =
      std::max(min_chunks, std::min(ntiles / 32, min_chunks + 8 * ((cap + per_chunk_wgs - 1) / per_chunk_wgs)));
  int best = min_chunks;
  long long best_cost = LLONG_MAX;
  for (int c = min_chunks; c <= max_chunks; ++c) {
    const long long rounds = ((long long)c * per_chunk_wgs + cap - 1) / cap;
    const long long cost = rounds * ((ntiles + c - 1) / c + kChunkOverhead);
    if (cost < best_cost) {
      best_cost = cost;
      best = c;
    }
  }
  return (ntiles + best - 1) / best;
}

hipError_t launch_nn(const NNArgs &args_in, hipStream_t stream) {
  NNArgs args = args_in;
  const int Npad = (args.N + 31) & ~31;
  // norms of the references; the same launch clears the keys (M <= N <= Npad)
  hipLaunchKernelGGL(k_nn_norms, dim3((Npad + 255) / 256, args.ndir), dim3(256), 0, stream, args);
  const int ntiles = Npad / 32;
  const int nqb = nn_qblocks(args.M);
  args.chunk_tiles = nn_chunk_tiles(ntiles, nqb * args.ndir);
  const int nchunk = nn_chunks(args.N, args.chunk_tiles);
  hipLaunchKernelGGL(k_nn, dim3(nqb * nchunk * args.ndir), dim3(64 * kWaves), 0, stream, args);
  return hipGetLastError();
}


hipError_t launch_gather_even(const uint8_t *desc1, uint8_t *out, int W, int H, hipStream_t stream) {
  const int n2 = ((W + 1) >> 1) * ((H + 1) >> 1);
  hipLaunchKernelGGL(k_gather_even, dim3((n2 + 255) / 256), dim3(256), 0, stream,
                     reinterpret_cast<const uint4 *>(desc1), reinterpret_cast<uint4 *>(out), W, H);
  return hipGetLastError();
}

hipError_t launch_remap_even(uint64_t *keys, int M, int W, hipStream_t stream) {
  hipLaunchKernelGGL(k_remap_even, dim3((M + 255) / 256), dim3(256), 0, stream, keys, M, W);
  return hipGetLastError();
}

size_t topl_scratch_bytes(int M) {
  return (((size_t)(kTopLMax - 1) * M * sizeof(uint64_t)) + 255) & ~(size_t)255;
}

hipError_t launch_topl(const TopLArgs &args_in, hipStream_t stream) {
  TopLArgs a = args_in;
  if (a.l < 1 || a.l > kTopLMax || a.M < 1 || a.N < 1) return hipErrorInvalidValue;
  NNArgs nn{};
  nn.ndir = a.ndir;
  nn.W = a.W;
  nn.H = a.H;
  nn.nc = a.nc;
  nn.Wc = a.Wc;
  nn.M = a.M;
  nn.N = a.N;
  const int ntiles = (a.N + 31) / 32;
  const int nqb = nn_qblocks(a.M);
  nn.chunk_tiles = nn_chunk_tiles(ntiles, nqb * a.ndir);
  const int nchunk = nn_chunks(a.N, nn.chunk_tiles);
  for (int k = 1; k < a.l; ++k) {
    TopLPrev prev{};
    for (int dr = 0; dr < a.ndir; ++dr) {
      const TopLDir &d = a.dir[dr];
      uint64_t *keys = d.keys + (size_t)(k - 1) * a.M;
      nn.dir[dr] = {d.Dq, d.Dr, const_cast<int32_t *>(d.nb), keys};
      prev.key[dr] = k == 1 ? d.nn_key : keys - a.M;
      hipError_t e = launch_fill_u64(keys, ~0ull, a.M, stream);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_nn_excl, dim3(nqb * nchunk * a.ndir), dim3(64 * kWaves), 0, stream, nn, prev);
  }
  hipLaunchKernelGGL(k_topl_assemble, dim3((a.M + 255) / 256, a.ndir), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace ffh
