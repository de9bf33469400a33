// Device helpers shared by the kernels: state pointer bundles, the tile map,
// corner-list staging and deterministic block reductions (DPP lane moves
// within 16-lane rows, then a fixed-order combine of the block's rows).
#pragma once

#include "pf_internal.hpp"

namespace pf {

template <typename T>
struct StateIn {
  const T* __restrict__ ux; const T* __restrict__ uy;
  const T* __restrict__ vx; const T* __restrict__ vy;
  const T* __restrict__ ax; const T* __restrict__ ay;
  const T* __restrict__ d;  const T* __restrict__ H;
};

template <typename T>
struct StateOut {
  T* __restrict__ ux; T* __restrict__ uy;
  T* __restrict__ vx; T* __restrict__ vy;
  T* __restrict__ ax; T* __restrict__ ay;
  T* __restrict__ d;  T* __restrict__ H;
};

template <typename T>
inline StateIn<T> state_in(const pf_state_t* s) {
  return StateIn<T>{(const T*)s->ux, (const T*)s->uy, (const T*)s->vx, (const T*)s->vy,
                    (const T*)s->ax, (const T*)s->ay, (const T*)s->d, (const T*)s->H};
}

template <typename T>
inline StateOut<T> state_out(pf_state_t* s) {
  return StateOut<T>{(T*)s->ux, (T*)s->uy, (T*)s->vx, (T*)s->vy, (T*)s->ax, (T*)s->ay, (T*)s->d, (T*)s->H};
}

// Tile processed by this workgroup.  Workgroups are handed to the chip's
// eight XCDs (each with its own L2) round-robin by workgroup id; this map
// gives XCD x the contiguous x-th eighth of the tile list, which is a compact
// region of the mesh (tiles are numbered in bisection order), so the halo
// nodes and elements that neighbouring tiles share are fetched into one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int tile_of_block(int n_tiles) {
  const int b = blockIdx.x;
  const int q = n_tiles / kXcds, rr = n_tiles % kXcds, x = b % kXcds, i = b / kXcds;
  return x * q + min(x, rr) + i;
}

// Stage the owned nodes' corner lists of a tile in LDS: offs[i] .. offs[i+1]
// index node i's entries of cl, which are tile-local corner ids 3 e + k in
// ascending element id.  Coalesced loads by the whole block; the caller
// synchronises before reading.
// Split staging: the loads of a tile's corner lists are issued into registers
// at kernel entry (NR row offsets and NC corner ids per thread) and stored to
// LDS later, so their latency overlaps the first phase's own loads; entries
// beyond the register capacity (large tiles) are copied at store time.
template <int NR, int NC>
struct StagedCorners {
  int32_t off[NR];
  uint16_t c[NC];
};

template <int NR, int NC>
__device__ __forceinline__ void stage_corners_load(const DevMesh& dm, const TileRec& t, StagedCorners<NR, NC>& s) {
  const int bs = blockDim.x;
#pragma unroll
  for (int u = 0; u < NR; ++u) s.off[u] = dm.lrow[t.node_begin + min(int(threadIdx.x) + u * bs, t.n_own)];
  const int last = t.n_corner - 1;   // every owned node has at least one corner
#pragma unroll
  for (int u = 0; u < NC; ++u) s.c[u] = dm.lcorner[t.corner_begin + min(int(threadIdx.x) + u * bs, last)];
}

template <int NR, int NC>
__device__ __forceinline__ void stage_corners_store(const DevMesh& dm, const TileRec& t,
                                                    const StagedCorners<NR, NC>& s, uint16_t* offs, uint16_t* cl) {
  const int bs = blockDim.x;
#pragma unroll
  for (int u = 0; u < NR; ++u) {
    const int i = threadIdx.x + u * bs;
    if (i <= t.n_own) offs[i] = uint16_t(s.off[u] - t.corner_begin);
  }
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    const int k = threadIdx.x + u * bs;
    if (k < t.n_corner) cl[k] = s.c[u];
  }
  for (int i = threadIdx.x + NR * bs; i <= t.n_own; i += bs)
    offs[i] = uint16_t(dm.lrow[t.node_begin + i] - t.corner_begin);
  for (int k = threadIdx.x + NC * bs; k < t.n_corner; k += bs) cl[k] = dm.lcorner[t.corner_begin + k];
}

// Each thread issues the loads of kStageBatch entries before it stores any of
// them, so a tile's lists arrive in a few memory round trips rather than one
// per block-wide stride (indices past the end are clamped to the last entry).
constexpr int kStageBatch = 8;
__device__ __forceinline__ void stage_corners(const DevMesh& dm, const TileRec& t, uint16_t* offs, uint16_t* cl) {
  const int bs = blockDim.x;
  for (int i0 = threadIdx.x; i0 <= t.n_own; i0 += kStageBatch * bs) {
    int32_t v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) v[u] = dm.lrow[t.node_begin + min(i0 + u * bs, t.n_own)];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (i0 + u * bs <= t.n_own) offs[i0 + u * bs] = uint16_t(v[u] - t.corner_begin);
  }
  const int last = t.n_corner - 1;
  for (int k0 = threadIdx.x; k0 < t.n_corner; k0 += kStageBatch * bs) {
    uint16_t v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) v[u] = dm.lcorner[t.corner_begin + min(k0 + u * bs, last)];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (k0 + u * bs < t.n_corner) cl[k0 + u * bs] = v[u];
  }
}

// Lane moves within 16-lane rows (DPP controls of the GFX9 family): swap
// neighbours, swap pairs, mirror each half-row, mirror the row.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- 7 - i within each 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <- 15 - i within each 16 lanes

template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(x));
  const int lo = __builtin_amdgcn_update_dpp(0, int(uint32_t(u)), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(uint32_t(u >> 32)), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(
      static_cast<long long>((static_cast<unsigned long long>(uint32_t(hi)) << 32) | uint32_t(lo)));
}

__device__ __forceinline__ double combine_op(uint32_t op, double s, double y) {
  return op == 0 ? s + y : (op == 1 ? fmin(s, y) : fmax(s, y));
}

// Reduce x over each 16-lane row: after the four steps every lane of a row
// holds the row's result (each step combines a lane with its mirror image, so
// both compute the same operation on the same pair).  All 64 lanes must be
// active.
template <uint32_t OP>
__device__ __forceinline__ double row_reduce(double x) {
  x = combine_op(OP, x, dpp_move<kDppXor1>(x));
  x = combine_op(OP, x, dpp_move<kDppXor2>(x));
  x = combine_op(OP, x, dpp_move<kDppHalfMirror>(x));
  x = combine_op(OP, x, dpp_move<kDppMirror>(x));
  return x;
}

template <int K, uint32_t OPS, int k = 0>
__device__ __forceinline__ void row_reduce_all(double (&v)[K]) {
  if constexpr (k < K) {
    v[k] = row_reduce<(OPS >> (2 * k)) & 3u>(v[k]);
    row_reduce_all<K, OPS, k + 1>(v);
  }
}

// Several block-wide reductions at once, without LDS shuffles: each value is
// reduced over every 16-lane row by DPP moves, lane 0 of each row stores the
// row's results, and thread k < K combines value k's 4 NW row results in a
// fixed order and returns it (other threads get 0).  OPS holds two bits per
// value: 0 sum, 1 min, 2 max.  Every thread of the block must call it; `sh`
// holds K * 4 * NW doubles and must not be in use by another reduction of the
// block.
template <int K, uint32_t OPS, int NW = kWaves>
__device__ __forceinline__ double block_reduce_rows(double (&v)[K], double* sh) {
  constexpr int R = 4 * NW;
  row_reduce_all<K, OPS>(v);
  const int lane = threadIdx.x & 63;
  if ((lane & 15) == 0) {
    const int r = (threadIdx.x >> 6) * 4 + (lane >> 4);
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k * R + r] = v[k];
  }
  __syncthreads();
  const int k = threadIdx.x;
  if (k >= K) return 0.0;
  const uint32_t op = (OPS >> (2 * k)) & 3u;
  double s = sh[k * R];
#pragma unroll
  for (int j = 1; j < R; ++j) s = combine_op(op, s, sh[k * R + j]);
  return s;
}

// Block-wide sum; every thread gets the result.  `sh` holds 4 kWaves doubles
// (one per 16-lane row); the rows' sums are added in a fixed order.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = row_reduce<0u>(v);
  const int lane = threadIdx.x & 63;
  __syncthreads();   // sh may still be read by a previous reduction
  if ((lane & 15) == 0) sh[(threadIdx.x >> 6) * 4 + (lane >> 4)] = v;
  __syncthreads();
  double s = sh[0];
#pragma unroll
  for (int j = 1; j < 4 * kWaves; ++j) s += sh[j];
  return s;
}

// Several block-wide reductions at once; only thread 0's v holds the block
// results afterwards.  Same scheme and arguments as block_reduce_rows.
template <int K, uint32_t OPS, int NW = kWaves>
__device__ __forceinline__ void block_reduce_to0(double (&v)[K], double* sh) {
  constexpr int R = 4 * NW;
  row_reduce_all<K, OPS>(v);
  const int lane = threadIdx.x & 63;
  if ((lane & 15) == 0) {
    const int r = (threadIdx.x >> 6) * 4 + (lane >> 4);
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k * R + r] = v[k];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t op = (OPS >> (2 * k)) & 3u;
    double t = sh[k * R];
#pragma unroll
    for (int j = 1; j < R; ++j) t = combine_op(op, t, sh[k * R + j]);
    v[k] = t;
  }
}

}  // namespace pf
