// nn_core.h -- exact nearest neighbour of up to 4 blocks of 16 query points
// against a prepared point cloud, one wavefront, on the gfx950 matrix cores.
//
// The squared distance |s - r|^2 = |s|^2 + (|r|^2 - 2 r.s); the first term is
// the same for every candidate r, so the argmin over r of eq. (1) is the
// argmin of the augmented dot product (-2r_x, -2r_y, -2r_z, |r|^2) . (s_x,
// s_y, s_z, 1): a K = 4 contraction, which is exactly the shape of one
// v_mfma_f32_16x16x4f32 (16 points x 16 queries per instruction).  The
// instruction's result equals, bit for bit, the chain of fused multiply-adds
// over the four products in order, so a lane can recompute any single
// candidate's value exactly and the index of the minimum is recovered
// without carrying it through the inner loop.
#pragma once
#include "asicp_internal.h"

namespace asicp {

// Prepared cloud: tile group tg (64 points, tg*64 .. tg*64+63) occupies 64
// float4; the float4 read by lane l holds component (l / 16) of the augmented
// points (tg*4 + u)*16 + (l % 16), u = 0..3.  This is the A-operand of four
// consecutive 16x16x4 MFMAs, so one coalesced 1 KiB wave load feeds them.
__device__ __forceinline__ void prep_store(float* prep_f, int m, float ax, float ay, float az, float an) {
  const int tg = m >> 6, u = (m >> 4) & 3, i = m & 15;
  float* base = prep_f + (size_t)tg * 256 + u;
  base[(0 * 16 + i) * 4] = ax;
  base[(1 * 16 + i) * 4] = ay;
  base[(2 * 16 + i) * 4] = az;
  base[(3 * 16 + i) * 4] = an;
}

// The prepared cloud as a raw buffer (gfx9 resource word 3 = 0x00020000):
// a tile group is read with a wave-uniform byte offset (scalar register) and
// the lane's 16-byte offset (vector register), the hardware's own address
// form, so no per-lane address arithmetic is spent in the scan loops.  The
// buffer's size bounds every read (out-of-range lanes would read zeros).
// The cloud is the same for the whole wavefront; reading the pointer and size
// from the first lane puts the resource in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t cloud_rsrc(const float4* __restrict__ prep, int ntg) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(prep);
  const unsigned long long lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
  const unsigned long long hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
  void* base = reinterpret_cast<void*>((hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, __builtin_amdgcn_readfirstlane(ntg) * 1024,
                                           0x00020000);
}

__device__ __forceinline__ float2 load_f2(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
  float2 f;
  __builtin_memcpy(&f, &v, 8);
  return f;
}

__device__ __forceinline__ float load_f1(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

__device__ __forceinline__ float4 load_tg(__amdgpu_buffer_rsrc_t r, int tg, unsigned lane_off) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, lane_off, tg * 1024, 0);
  float4 f;
  __builtin_memcpy(&f, &v, 16);
  return f;
}

// Chunk = CH tile groups (CH = 1 or 2: 64 or 128 points), the unit of
// spatial pruning; the scans below take CH as a template argument (the
// forward NN's is a launch choice; the contact clouds of the reverse NN use
// kChunkTG).  Prepared clouds are padded to a multiple of 256 points, a
// whole number of chunk pairs for either size, so the full scan's loop runs
// without a tail.
constexpr int kChunkTG = 2;
constexpr int kPadPoints = 256;

// Fold the 16 distances a lane holds for one query and one tile group into
// its running minimum: one v_min3 per two distances (the floor for a
// min-reduction; on gfx950 VALU work does not overlap the matrix core).
template <int Q>
__device__ __forceinline__ void tile_group(const float4& a, const float* b, float* m,
                                           const bool* need = nullptr) {
  const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (need && !need[q]) continue;  // wave-uniform
    const f4v d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b[q], zero, 0, 0, 0);
    const f4v d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b[q], zero, 0, 0, 0);
    const f4v d2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b[q], zero, 0, 0, 0);
    const f4v d3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b[q], zero, 0, 0, 0);
    float r = m[q];
    r = fminf(fminf(r, d0[0]), d0[1]);
    r = fminf(fminf(r, d0[2]), d0[3]);
    r = fminf(fminf(r, d1[0]), d1[1]);
    r = fminf(fminf(r, d1[2]), d1[3]);
    r = fminf(fminf(r, d2[0]), d2[1]);
    r = fminf(fminf(r, d2[2]), d2[3]);
    r = fminf(fminf(r, d3[0]), d3[1]);
    r = fminf(fminf(r, d3[2]), d3[3]);
    m[q] = r;
  }
}

// Fold one chunk (CH tile groups) into each lane's running minimum.  The
// chunk's own minimum is folded first, so that the chunk recorded with the
// running minimum is the lowest-index chunk holding it whatever order the
// chunks are visited in: a chunk with a smaller value replaces it, one with
// an equal value only if its index is lower.  ASCENDING (the full scan, which
// visits chunks in index order) records a chunk only if its value is
// smaller, which selects the same chunk, and keeps one tile group's MFMA
// results live at a time (fewer registers, so more wavefronts per SIMD hide
// the matrix-core latency).
template <int Q, int CH, bool ASCENDING = false>
__device__ __forceinline__ void chunk_step(const float4 (&a)[CH], const float* b, float* best, int* bch,
                                           int c, const bool* need = nullptr) {
  float m[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) m[q] = __builtin_inff();
#pragma unroll
  for (int t = 0; t < CH; ++t) {
    if (ASCENDING && t) __builtin_amdgcn_sched_barrier(0);
    tile_group<Q>(a[t], b, m, need);
  }
  // A block the chunk was not compared with keeps m = +inf, and its running
  // minimum is finite (the first chunk is compared with every block), so the
  // updates below leave it as it is.
  if (ASCENDING) {
#pragma unroll
    for (int q = 0; q < Q; ++q) bch[q] = m[q] < best[q] ? c : bch[q];
  } else {
    // A chunk value equal to the running minimum (a tie across chunks) is
    // rare: one wave-wide test, and only then the lower-index rule
    bool tie = false;
#pragma unroll
    for (int q = 0; q < Q; ++q) tie = tie || m[q] == best[q];
    if (__ballot(tie) != 0ull) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
        bch[q] = (m[q] < best[q] || (m[q] == best[q] && c < bch[q])) ? c : bch[q];
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) bch[q] = m[q] < best[q] ? c : bch[q];
    }
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) best[q] = fminf(best[q], m[q]);
}

// Re-find the index of each query's minimum.  Each lane group owns rows
// 4*grp .. 4*grp+3 of every 16-point tile and knows its minimum and the chunk
// where its running minimum last decreased.  Among the lane groups reaching
// the query's minimum, the one with the lowest such chunk is chosen, and the
// lowest index in that chunk holding the minimal value is returned; candidate
// values are recomputed with the exact fused multiply-add chain the MFMA
// performs.
//
// With BATCH, when one lane group wins (the usual case), the query's four
// lanes test that group's 4 rows in all 4 CH tiles of the chunk: lane
// group g takes tiles g CH .. g CH + CH - 1 (sub-tiles of
// one tile group, adjacent in the prepared cloud), so 16 buffer loads with
// immediate offsets fetch all operands at once; qc holds the lane's query
// (x, y, z per block) from the caller, or is null (then the query is read
// from the B operand's rows).  Otherwise (or on ties between lane
// groups, which test all 16 rows) the lanes split the tiles and test row by
// row, reading the query from the B operand.
template <int Q, bool BATCH, int CH>
__device__ __forceinline__ void nn_rescan(const float4* __restrict__ prep, __amdgpu_buffer_rsrc_t rs,
                                          const float* b, const float* qc, const float* best,
                                          const int* bch, int* idx, int32_t* miss) {
  const int lane = lane_id();
  const int grp = lane >> 4;
  const float* pf = reinterpret_cast<const float*>(prep);
  const int j = lane & 15;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const float v = best[q];
    const float vmin = rows_min(v);
    const int cmin = rows_min_i((v == vmin) ? bch[q] : 0x7fffffff);
    const bool mine = (v == vmin) && (bch[q] == cmin);
    const int gw = rows_min_i(mine ? grp : 4);
    const int ng = rows_sum_i(mine ? 1 : 0);
    int cand = 0x7fffffff;
    if (cmin != 0x7fffffff) {
      if (BATCH && ng == 1) {
        // the lane's query (x, y, z): kept by the caller, or gathered from
        // rows 0-2 of the B operand
        const float s0 = qc ? qc[3 * q] : __shfl(b[q], j, 64);
        const float s1 = qc ? qc[3 * q + 1] : __shfl(b[q], j + 16, 64);
        const float s2 = qc ? qc[3 * q + 2] : __shfl(b[q], j + 32, 64);
        const int t0 = grp * CH;  // first tile of the lane group within the chunk
        const int tgi = t0 >> 2, u0 = t0 & 3, r0 = 4 * gw;
        const unsigned voff = 4u * (unsigned)((cmin * CH + tgi) * 256 + r0 * 4 + u0);
        float a[4][4][CH];  // [component][row][sub-tile]
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) {
            if (CH == 2) {
              const float2 v = load_f2(rs, voff + 16u * (unsigned)(k * 16 + ii));
              a[k][ii][0] = v.x;
              a[k][ii][CH - 1] = v.y;
            } else {
              a[k][ii][0] = load_f1(rs, voff + 16u * (unsigned)(k * 16 + ii));
            }
          }
        const int tbase = (cmin * CH * 4 + t0) * 16 + r0;
#pragma unroll
        for (int u = CH - 1; u >= 0; --u)
#pragma unroll
          for (int ii = 3; ii >= 0; --ii) {  // the lowest index is tested last, so it wins
            float acc = __builtin_fmaf(a[0][ii][u], s0, 0.0f);
            acc = __builtin_fmaf(a[1][ii][u], s1, acc);
            acc = __builtin_fmaf(a[2][ii][u], s2, acc);
            acc = __builtin_fmaf(a[3][ii][u], 1.0f, acc);
            if (acc == vmin) cand = tbase + 16 * u + ii;
          }
      } else {
        const float s0 = __shfl(b[q], j, 64);
        const float s1 = __shfl(b[q], j + 16, 64);
        const float s2 = __shfl(b[q], j + 32, 64);
        const float s3 = __shfl(b[q], j + 48, 64);
        const int r0 = (ng > 1) ? 0 : 4 * gw, r1 = (ng > 1) ? 16 : 4 * gw + 4;
        for (int tt = 0; tt < CH && cand == 0x7fffffff; ++tt) {
          const int t = grp + 4 * tt;  // tile within the chunk: tile group t/4, sub-tile t%4
          const float* base = pf + (size_t)(cmin * CH + (t >> 2)) * 256 + (t & 3);
          for (int i = r0; i < r1; ++i) {
            float acc = __builtin_fmaf(base[(0 * 16 + i) * 4], s0, 0.0f);
            acc = __builtin_fmaf(base[(1 * 16 + i) * 4], s1, acc);
            acc = __builtin_fmaf(base[(2 * 16 + i) * 4], s2, acc);
            acc = __builtin_fmaf(base[(3 * 16 + i) * 4], s3, acc);
            if (acc == vmin) {
              cand = ((cmin * CH + (t >> 2)) * 4 + (t & 3)) * 16 + i;
              break;
            }
          }
        }
      }
    }
    cand = rows_min_i(cand);
    if (cand == 0x7fffffff) {
      if (lane == 0) atomicOr(miss, 1);
      cand = 0;
    }
    idx[q] = cand;
  }
}

// Q blocks of 16 queries.  Lane l supplies bq[q] = component (l / 16) of the
// augmented query (s_x, s_y, s_z, 1) number (l % 16) of block q.  `ntg` (a
// multiple of 4) tile groups of the prepared cloud are scanned in order.  On
// return every lane holds in idx[q] the index (0 .. 64*ntg-1) of the nearest
// point for query (l % 16) of block q: the lowest index among the candidates
// with the smallest FP32 value.  A query whose minimum cannot be re-found
// (only possible with non-finite inputs) gets index 0 and sets *miss.
// qc[3q + a] = component a of the lane's query (l % 16) of block q, or null
// (the re-scan then reads the queries from the B operand).
template <int Q, int CH>
__device__ __forceinline__ void nn_scan(const float4* __restrict__ prep, int ntg, const float* bq,
                                        const float* qc, int* idx, int32_t* miss) {
  const int lane = lane_id();
  float b[Q], best[Q];
  int bch[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    b[q] = bq[q];
    best[q] = __builtin_inff();
    bch[q] = 0;
  }
  const int nch = ntg / CH;  // even
  const unsigned lo = 16u * (unsigned)lane;
  const __amdgpu_buffer_rsrc_t rs = cloud_rsrc(prep, ntg);
  float4 x[CH], y[CH];
#pragma unroll
  for (int t = 0; t < CH; ++t) x[t] = load_tg(rs, t, lo);
  for (int c = 0; c < nch; c += 2) {
#pragma unroll
    for (int t = 0; t < CH; ++t) y[t] = load_tg(rs, (c + 1) * CH + t, lo);
    chunk_step<Q, CH, true>(x, b, best, bch, c);
    if (c + 2 < nch) {
#pragma unroll
      for (int t = 0; t < CH; ++t) x[t] = load_tg(rs, (c + 2) * CH + t, lo);
    }
    chunk_step<Q, CH, true>(y, b, best, bch, c + 1);
  }
  nn_rescan<Q, true, CH>(prep, rs, b, qc, best, bch, idx, miss);
}

// Q non-negative floats packed as FP16 pairs with rounding toward zero, so an
// unpacked value never exceeds the original (lower bounds stay lower bounds;
// +inf stays +inf).
template <int Q>
struct LbPack {
  __attribute__((ext_vector_type(2))) __fp16 h[(Q + 1) / 2];
  __device__ __forceinline__ void set(int q, float v) {
    if (q & 1) h[q >> 1] = __builtin_amdgcn_cvt_pkrtz(h[q >> 1][0], v);
    else h[q >> 1] = __builtin_amdgcn_cvt_pkrtz(v, 0.0f);
  }
  __device__ __forceinline__ float get(int q) const { return (float)h[q >> 1][q & 1]; }
};

// Chunk boxes as a raw buffer (like cloud_rsrc): box c is read with the
// lane's 32-bit byte offset c * 32, no 64-bit address per lane; boxes beyond
// the buffer read as zeros.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t box_rsrc(const float* __restrict__ box, int nch) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(box);
  const unsigned long long lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)a);
  const unsigned long long hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(a >> 32));
  void* base = reinterpret_cast<void*>((hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, __builtin_amdgcn_readfirstlane(nch) * 32, 0x00020000);
}

__device__ __forceinline__ void load_box(__amdgpu_buffer_rsrc_t r, int c, float bx[8]) {
  const auto a = __builtin_amdgcn_raw_buffer_load_b128(r, (unsigned)c * 32u, 0, 0);
  const auto b = __builtin_amdgcn_raw_buffer_load_b128(r, (unsigned)c * 32u + 16u, 0, 0);
  __builtin_memcpy(bx, &a, 16);
  __builtin_memcpy(bx + 4, &b, 16);
}

// Squared distance from the box [lo, hi] to the box [qlo, qhi] (0 if they
// overlap): a lower bound of |s - r|^2 for any query s in the query box and
// any point r in the chunk box.
__device__ __forceinline__ float box_gap2(const float* bx, const float qlo[3], const float qhi[3]) {
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float g = fmaxf(fmaxf(bx[a] - qhi[a], qlo[a] - bx[4 + a]), 0.f);
    s = __builtin_fmaf(g, g, s);
  }
  return s;
}

// Squared distance from point p to the box [bx[0..2], bx[4..6]] (0 inside).
__device__ __forceinline__ float point_box2(const float* p, const float* bx) {
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float g = fmaxf(fmaxf(bx[a] - p[a], p[a] - bx[4 + a]), 0.f);
    s = __builtin_fmaf(g, g, s);
  }
  return s;
}

// As nn_scan, but a chunk is only compared with a block of 16 queries if the
// chunk's box can hold a point nearer than the block's current worst bound:
// exact (the same nearest distances as scanning everything).  Queries must be
// spatially coherent for this to pay (contact clouds are in k-d leaf order).
//
// The chunk nearest to the wave's query box is scanned first; the other
// candidates follow nearest first (smallest box-to-box lower bound over the
// blocks that may need them), and the scan of a 64-chunk block stops once
// every remaining lower bound exceeds every block's bound.  A block of
// queries takes a candidate chunk only while the box-to-box lower bound is
// within the block's bound (refreshed every ASICP_NN_REFRESH chunks) and,
// with FINE, only if some query's point-to-box distance is within that
// query's own best.  None of these tests can drop
// a chunk holding a value equal to a final minimum, and the chunk record of
// chunk_step does not depend on the visiting order, so the results do not
// depend on them.
// snorm[q] = |s|^2 of the lane's query in block q (turns the reduced value
// |r|^2 - 2 r.s into a squared distance).  With OWN the lane instead owns one
// query, number (l % 16) of block min(l / 16, Q - 1), whose coordinates the
// caller passes in own[3]: the bounds and the per-query chunk test are then
// computed once per lane for all blocks at once (one lane per query rather
// than four copies of each block), |s|^2 comes from own, snorm may be null,
// and the re-scan reads the queries from the B operand.  box = the cloud's
// chunk boxes;
// blk_box = the box of every block of 64 chunks, or null (no block test);
// m = real points of the cloud; vq[q] = real queries of block q; r2max = the
// largest |r|^2 of the cloud.  Returns the number of (query, point) distances
// evaluated (wave-uniform).  Every bound carries a slack for the FP32
// rounding of the distances it is compared with: 1e-4 relative, plus
// 5e-7 (r2max + |s|^2) (the rounding of the fused chain |r|^2 - 2 r.s is
// at most a few units of 2^-24 times |r|^2 + 2 |r| |s| <= 2 (|r|^2 + |s|^2)),
// plus 1e-7 (squared length units).
template <int Q, bool OWN, bool FINE, int CH>
__device__ __forceinline__ long long nn_scan_pruned(const float4* __restrict__ prep, int ntg, int m,
                                                    const float* __restrict__ box,
                                                    const float* __restrict__ blk_box, const float* bq,
                                                    const float* snorm, const float* own, const int* vq,
                                                    float r2max, int* idx, int32_t* miss) {
  static_assert(OWN || !FINE, "the per-query chunk test needs the lane's own query");
  const int lane = lane_id();
  const int qo = min(lane >> 4, Q - 1);  // with OWN: the block of the lane's own query
  float b[Q], best[Q];
  int bch[Q];
  float qlo[Q][3], qhi[Q][3];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    b[q] = bq[q];
    best[q] = __builtin_inff();
    bch[q] = 0;
    // block q's query box: row a of the lanes holds component a
    const float lo = row_min(bq[q]), hi = row_max(bq[q]);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      qlo[q][a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(lo), 16 * a));
      qhi[q][a] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(hi), 16 * a));
    }
  }
  const int nch = ntg / CH;
  const unsigned lo = 16u * (unsigned)lane;
  const __amdgpu_buffer_rsrc_t rs = cloud_rsrc(prep, ntg);
  // qbo (OWN): the lane's own query's current best squared distance, with
  // slack; ub[q]: the largest such bound over block q's queries
  float ub[Q], qbo = 0.0f, ubmax;
  auto refresh = [&]() {
    if (OWN) {
      float mn = rows_min(best[0]);
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        const float v = rows_min(best[q]);
        mn = qo == q ? v : mn;
      }
      // |s|^2 from the query's coordinates, recomputed here rather than kept
      // in a register through the scan (the empty constraints keep the
      // compiler from hoisting it out of the loop)
      float x = own[0], y = own[1], z = own[2];
      __asm__("" : "+v"(x), "+v"(y), "+v"(z));
      const float sn = __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x));
      qbo = __builtin_fmaf(mn + sn, 1.0001f, __builtin_fmaf(5e-7f, r2max + sn, 1e-7f));
      // row q holds block q's queries
      const float rm = row_max(qbo);
#pragma unroll
      for (int q = 0; q < Q; ++q) ub[q] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rm), 16 * q));
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const float sn = snorm[q];
        const float qb = __builtin_fmaf(rows_min(best[q]) + sn, 1.0001f, __builtin_fmaf(5e-7f, r2max + sn, 1e-7f));
        // every row holds the same 16 queries, so the row maximum is uniform
        ub[q] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(row_max(qb))));
      }
    }
    ubmax = ub[0];
#pragma unroll
    for (int q = 1; q < Q; ++q) ubmax = fmaxf(ubmax, ub[q]);
  };
  // nearest chunk to the union of the blocks' boxes
  float ulo[3], uhi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    ulo[a] = qlo[0][a];
    uhi[a] = qhi[0][a];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      ulo[a] = fminf(ulo[a], qlo[q][a]);
      uhi[a] = fmaxf(uhi[a], qhi[q][a]);
    }
  }
  // (smallest gap, then lowest index; gaps are non-negative, so their bit
  // patterns order like their values; a lane without a chunk never wins)
  const __amdgpu_buffer_rsrc_t rb = box_rsrc(box, nch);
  unsigned gbest = 0xffffffffu;
  int cbest = 0x7fffffff;
  for (int c = lane; c < nch; c += 64) {
    float cb[8];
    load_box(rb, c, cb);
    const unsigned g = __float_as_uint(box_gap2(cb, ulo, uhi));
    if (c == lane || g < gbest) {
      gbest = g;
      cbest = c;
    }
  }
  // lane b: the lower bound between the union box and block b's box (the
  // first 64 blocks of 64 chunks; later blocks are not tested)
  float blk_gap = 0.0f;
  if (blk_box && nch > 64 && lane < ((nch + 63) >> 6)) {
    float bb[8];
    load_box(box_rsrc(blk_box, (nch + 63) >> 6), lane, bb);
    blk_gap = box_gap2(bb, ulo, uhi);
  }
  const unsigned gmin = wave_min_u(gbest);
  const int c0 = __builtin_amdgcn_readfirstlane(
      min((int)wave_min_u(gbest == gmin ? (unsigned)cbest : 0x7fffffffu), nch - 1));  // same in every lane
  // pair count (a statistic): every operand is wave-uniform, so it stays in
  // scalar registers
  const int mu = __builtin_amdgcn_readfirstlane(m);
  int vqu[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) vqu[q] = __builtin_amdgcn_readfirstlane(vq[q]);
  long long pairs = 0;
  {
    const int pts = max(0, min((64 * CH), mu - (64 * CH) * c0));
    float4 x0[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) x0[t] = load_tg(rs, c0 * CH + t, lo);
    chunk_step<Q, CH>(x0, b, best, bch, c0);
#pragma unroll
    for (int q = 0; q < Q; ++q) pairs += (long long)(pts * vqu[q]);
  }
  refresh();
  int since = 0;
  for (int blk = 0; blk < nch; blk += 64) {
    // the whole block of 64 chunks is skipped when its box is beyond every
    // block's bound: each chunk box lies in the block box and each block of
    // queries in the union box, so no chunk of it could be a candidate
    if (blk_box && nch > 64 && blk < 64 * 64 &&
        __int_as_float(__builtin_amdgcn_readlane(__float_as_int(blk_gap), blk >> 6)) > ubmax)
      continue;
    const int c = blk + lane;
    // lb(q): lower bound of the squared distance between block q's queries
    // and the lane's chunk, kept as FP16 pairs rounded toward zero (still
    // lower bounds, in half the registers)
    LbPack<Q> lbp;
    // in[q]: the lane's chunk may still be needed by block q of the queries;
    // mq[q]: the same as a wave-uniform mask over the 64 chunks of the block
    bool in[Q];
    unsigned long long mq[Q];
    float cb[8];
    load_box(rb, c, cb);  // zeros beyond the last chunk (not used there)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float g = c < nch ? box_gap2(cb, qlo[q], qhi[q]) : __builtin_inff();
      lbp.set(q, g);
      in[q] = c < nch && c != c0 && g <= ub[q];
      mq[q] = __ballot(in[q]);
    }
    auto lb = [&](int q) { return lbp.get(q); };
    // Candidates are visited nearest first: the key of the lane's chunk is its
    // smallest lower bound over the blocks that may need it, with the lane in
    // the low 6 bits (unique keys, rounded down, so the exit test below stays
    // conservative).  Taken chunks and chunks no block needs have no key.
    bool taken = false;
    auto key_of = [&]() -> unsigned {
      float k = __builtin_inff();
#pragma unroll
      for (int q = 0; q < Q; ++q) k = in[q] ? fminf(k, lb(q)) : k;
      return (taken || !(k < __builtin_inff())) ? 0xffffffffu : ((__float_as_uint(k) & ~63u) | (unsigned)lane);
    };
    unsigned key = key_of();
    // the next chunk, or -1 once every remaining lower bound exceeds every
    // block's bound (then no remaining chunk can hold a nearer point)
    auto pick = [&]() -> int {
      const unsigned mk = __builtin_amdgcn_readfirstlane(wave_min_u(key));
      if (mk == 0xffffffffu || __uint_as_float(mk & ~63u) > ubmax) return -1;
      const int l = (int)(mk & 63u);
      taken = taken || lane == l;
      key = lane == l ? 0xffffffffu : key;
      return l;
    };
    int cl = pick();
    if (cl < 0) continue;
    // One step compares chunk cl (held in cur) and loads the next candidate
    // into nxt while it does; two steps per iteration swap the roles of the
    // register pairs, so no copy is made between them.
    float4 x[CH], y[CH];
    auto fetch = [&](float4 (&dst)[CH], int l) {
#pragma unroll
      for (int t = 0; t < CH; ++t) dst[t] = load_tg(rs, (blk + l) * CH + t, lo);
    };
    fetch(x, cl);
    auto step = [&](const float4 (&cur)[CH], float4 (&nxt)[CH]) {
      const int cc = blk + cl;
      int nl = pick();
      if (nl >= 0) fetch(nxt, nl);
      const int pts = max(0, min((64 * CH), mu - (64 * CH) * cc));
      // block q is compared only if chunk cc is still in its mask (a scalar
      // bit test) and, with FINE, some query of the block may improve
      bool need[Q], any = false;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        need[q] = (mq[q] >> cl) & 1ull;
        any = any || need[q];
      }
      if (FINE && any) {
        // one test per lane's own query; bits 16q .. 16q + 15 are block q's
        const unsigned long long fm = __ballot(point_box2(own, box + (size_t)cc * 8) <= qbo);
#pragma unroll
        for (int q = 0; q < Q; ++q) need[q] = need[q] && ((fm >> (16 * q)) & 0xffffull) != 0ull;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) pairs += need[q] ? (long long)(pts * vqu[q]) : 0ll;
      chunk_step<Q, CH>(cur, b, best, bch, cc, need);
      if (++since == ASICP_NN_REFRESH) {
        since = 0;
        refresh();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          in[q] = in[q] && lb(q) <= ub[q];
          mq[q] = __ballot(in[q]);
        }
        // the prefetched chunk stays taken; the rest are re-keyed
        if (nl >= 0) {
          const bool was = lane == nl;
          taken = taken && !was;
          key = key_of();
          const int n2 = pick();
          if (n2 != nl) {  // the prefetched chunk is no longer the nearest needed one
            if (was) key = key_of();  // hand it back to the pool
            nl = n2;
            if (nl >= 0) fetch(nxt, nl);
          }
        } else {
          key = key_of();
        }
      }
      cl = nl;
    };
    while (cl >= 0) {
      step(x, y);
      if (cl < 0) break;
      step(y, x);
    }
  }
  nn_rescan<Q, OWN, CH>(prep, rs, b, nullptr, best, bch, idx, miss);
  return pairs;
}

}  // namespace asicp
