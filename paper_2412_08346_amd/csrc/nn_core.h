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

__device__ __forceinline__ float min16(const f4v& a, const f4v& b, const f4v& c, const f4v& d) {
  float m = fminf(fminf(a[0], a[1]), a[2]);
  m = fminf(fminf(m, a[3]), b[0]);
  m = fminf(fminf(m, b[1]), b[2]);
  m = fminf(fminf(m, b[3]), c[0]);
  m = fminf(fminf(m, c[1]), c[2]);
  m = fminf(fminf(m, c[3]), d[0]);
  m = fminf(fminf(m, d[1]), d[2]);
  return fminf(m, d[3]);
}

// Q blocks of 16 queries.  Lane l supplies bq[q] = component (l / 16) of the
// augmented query (s_x, s_y, s_z, 1) number (l % 16) of block q.  On return,
// every lane holds in idx[q] the index (0 .. 64*ntg-1) of the nearest point
// for query (l % 16) of block q: the lowest index among the candidates with
// the smallest FP32 value.  A query whose minimum cannot be re-found (only
// possible with non-finite inputs) gets index 0 and sets *miss.
template <int Q>
__device__ __forceinline__ void nn_scan(const float4* __restrict__ prep, int ntg, const float* bq,
                                        int* idx, int32_t* miss) {
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 4;
  const f4v zero = {0.0f, 0.0f, 0.0f, 0.0f};
  float b[Q], best[Q];
  int bchunk[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    b[q] = bq[q];
    best[q] = __builtin_inff();
    bchunk[q] = 0;
  }
  float4 a0 = prep[lane];
  float4 a1 = (ntg > 1) ? prep[64 + lane] : a0;
  for (int tg = 0; tg < ntg; ++tg) {
    float4 a2 = a1;
    if (tg + 2 < ntg) a2 = prep[(size_t)(tg + 2) * 64 + lane];
    f4v acc[Q][4];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      acc[q][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.x, b[q], zero, 0, 0, 0);
      acc[q][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.y, b[q], zero, 0, 0, 0);
      acc[q][2] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.z, b[q], zero, 0, 0, 0);
      acc[q][3] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0.w, b[q], zero, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float m = min16(acc[q][0], acc[q][1], acc[q][2], acc[q][3]);
      if (m < best[q]) {
        best[q] = m;
        bchunk[q] = tg;
      }
    }
    a0 = a1;
    a1 = a2;
  }
  // Re-find the index: each lane group owns rows 4*grp .. 4*grp+3 of every
  // tile; the earliest tile group holding its minimum is bchunk.
  const float* pf = reinterpret_cast<const float*>(prep);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const float v = best[q];
    float vmin = fminf(v, __shfl_xor(v, 16, 64));
    vmin = fminf(vmin, __shfl_xor(vmin, 32, 64));
    const int j = lane & 15;
    const float s0 = __shfl(b[q], j, 64);
    const float s1 = __shfl(b[q], j + 16, 64);
    const float s2 = __shfl(b[q], j + 32, 64);
    const float s3 = __shfl(b[q], j + 48, 64);
    int cand = 0x7fffffff;
    if (v == vmin) {
      const float* base = pf + (size_t)bchunk[q] * 256;
      for (int u = 0; u < 4 && cand == 0x7fffffff; ++u) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * grp + r;
          const float c0 = base[(0 * 16 + i) * 4 + u];
          const float c1 = base[(1 * 16 + i) * 4 + u];
          const float c2 = base[(2 * 16 + i) * 4 + u];
          const float c3 = base[(3 * 16 + i) * 4 + u];
          float acc = __builtin_fmaf(c0, s0, 0.0f);
          acc = __builtin_fmaf(c1, s1, acc);
          acc = __builtin_fmaf(c2, s2, acc);
          acc = __builtin_fmaf(c3, s3, acc);
          if (acc == v && cand == 0x7fffffff) cand = (bchunk[q] * 4 + u) * 16 + i;
        }
      }
    }
    cand = min(cand, __shfl_xor(cand, 16, 64));
    cand = min(cand, __shfl_xor(cand, 32, 64));
    if (cand == 0x7fffffff) {
      if (j == 0 && grp == 0) atomicOr(miss, 1);
      cand = 0;
    }
    idx[q] = cand;
  }
}

}  // namespace asicp
