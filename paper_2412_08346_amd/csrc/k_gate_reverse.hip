// k_gate_reverse.hip -- SDF collision gate and reverse nearest neighbour
// (Sec. IV-C and eq. (18); Algorithm 1's collision branch).
//
// One workgroup = one particle x 256 points of its collision cloud.  Each
// point is moved into the gripper frame, c' = R^T (c - t), and looked up in
// the preshape's SDF by trilinear interpolation; it collides when it lies in
// the node box and the value is strictly negative.  Colliding points are
// compacted in index order and paired with their nearest contact point, in
// the gripper frame (a rigid motion preserves distances, so this is the
// nearest transformed contact point of eq. (18)).  Partial sums, gripper
// frame: [sum |s - c'|^2, sum (s - c') (3), sum s x (s - c') (3), count].
#include "nn_core.h"

namespace asicp {

__device__ __forceinline__ int xcd_logical_g(int b, int nwg) {
  const int per = (nwg + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ bool sdf_collides(const PreInfo& pi, float px, float py, float pz) {
  const float ux = (px - pi.ox) * pi.inv_cell;
  const float uy = (py - pi.oy) * pi.inv_cell;
  const float uz = (pz - pi.oz) * pi.inv_cell;
  if (!(ux >= 0.f && ux <= (float)(pi.nx - 1) && uy >= 0.f && uy <= (float)(pi.ny - 1) &&
        uz >= 0.f && uz <= (float)(pi.nz - 1)))
    return false;
  const int ix = min((int)floorf(ux), pi.nx - 2);
  const int iy = min((int)floorf(uy), pi.ny - 2);
  const int iz = min((int)floorf(uz), pi.nz - 2);
  const float fx = ux - (float)ix, fy = uy - (float)iy, fz = uz - (float)iz;
  const size_t sx = 1, sy = (size_t)pi.nx, sz = (size_t)pi.nx * pi.ny;
  const float* v = pi.sdf + (size_t)iz * sz + (size_t)iy * sy + ix;
  const float c00 = (1.f - fx) * v[0] + fx * v[sx];
  const float c10 = (1.f - fx) * v[sy] + fx * v[sy + sx];
  const float c01 = (1.f - fx) * v[sz] + fx * v[sz + sx];
  const float c11 = (1.f - fx) * v[sz + sy] + fx * v[sz + sy + sx];
  const float c0 = (1.f - fy) * c00 + fy * c10;
  const float c1 = (1.f - fy) * c01 + fy * c11;
  return (1.f - fz) * c0 + fz * c1 < 0.f;
}

template <int Q>
__device__ __forceinline__ void rev_scan(const Dev& d, const PreInfo& pi, const float* bq, int* idx) {
  nn_scan<Q>(d.pre_prep + (size_t)pi.prep_tg_begin * 64, pi.ntg, bq, idx, d.flags + 1);
}

__global__ __launch_bounds__(256) void k_gate_reverse(Dev d) {
  __shared__ float lx[kGateChunk], ly[kGateChunk], lz[kGateChunk];
  __shared__ int lm[kGateChunk];
  __shared__ int wcount[4];
  __shared__ float wpart[4][kPartStride];

  const int nwg = d.total_gate_wgs;
  const int logical = xcd_logical_g(blockIdx.x, nwg);
  if (logical >= nwg) return;  // uniform over the workgroup
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  int lo = 0, hi = d.G - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.groups[mid].gate_off <= logical) lo = mid; else hi = mid - 1;
  }
  const GroupInfo gi = d.groups[lo];
  const PreInfo& pi = d.pres[gi.pre];
  const ObjInfo& oi = d.objs[gi.obj];
  const int local = logical - gi.gate_off;
  const int pj = local / oi.gate_chunks, cc = local - pj * oi.gate_chunks;
  const int i = lo * d.K + pj;

  float t[3], qv[4], R[9];
  load_pose(d.theta, d.Ktot, i, t, qv);
  quat_to_rot(qv[0], qv[1], qv[2], qv[3], R);

  const int m = cc * kGateChunk + tid;
  bool col = false;
  float px = 0.f, py = 0.f, pz = 0.f;
  if (m < oi.mc) {
    const float dx = d.cx[oi.c_begin + m] - t[0];
    const float dy = d.cy[oi.c_begin + m] - t[1];
    const float dz = d.cz[oi.c_begin + m] - t[2];
    px = R[0] * dx + R[3] * dy + R[6] * dz;
    py = R[1] * dx + R[4] * dy + R[7] * dz;
    pz = R[2] * dx + R[5] * dy + R[8] * dz;
    col = sdf_collides(pi, px, py, pz);
    if (d.dbg_rev && !col) d.dbg_rev[(size_t)i * d.mc_max + m] = -1;
  }
  const unsigned long long mask = __ballot(col);
  const int before = __popcll(mask & ((1ull << lane) - 1ull));
  if (lane == 0) wcount[w] = __popcll(mask);
  __syncthreads();
  int base = 0, total = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    base += (k < w) ? wcount[k] : 0;
    total += wcount[k];
  }
  if (col) {
    const int pos = base + before;
    lx[pos] = px; ly[pos] = py; lz[pos] = pz; lm[pos] = m;
  }
  __syncthreads();

  float* out = d.col_part + ((size_t)i * d.max_gate_chunks + cc) * kPartStride;
  if (total == 0) {
    if (tid < kPartStride) out[tid] = 0.f;
    return;
  }
  // reverse NN: blocks of 16 colliding points, block b handled by wave b % 4
  const int nb = (total + 15) >> 4;
  const int nbw = (nb > w) ? (nb - w + 3) >> 2 : 0;
  float e2 = 0.f, ex = 0.f, ey = 0.f, ez = 0.f, mx = 0.f, my = 0.f, mz = 0.f;
  if (nbw > 0) {
    const int comp = lane >> 4;
    float bq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pos = (w + 4 * q) * 16 + (lane & 15);
      float v = 0.f;
      if (q < nbw && pos < total) v = comp == 0 ? lx[pos] : comp == 1 ? ly[pos] : lz[pos];
      bq[q] = comp == 3 ? 1.0f : v;
    }
    int idx[4] = {0, 0, 0, 0};
    switch (nbw) {
      case 1: rev_scan<1>(d, pi, bq, idx); break;
      case 2: rev_scan<2>(d, pi, bq, idx); break;
      case 3: rev_scan<3>(d, pi, bq, idx); break;
      default: rev_scan<4>(d, pi, bq, idx); break;
    }
    int my_idx = idx[0];
    if (comp == 1) my_idx = idx[1];
    if (comp == 2) my_idx = idx[2];
    if (comp == 3) my_idx = idx[3];
    const int pos = (w + 4 * comp) * 16 + (lane & 15);
    if (comp < nbw && pos < total) {
      if (my_idx >= pi.n) {
        atomicOr(d.flags + 1, 4);
        my_idx = pi.n - 1;
      }
      const float sx = d.sx[pi.s_begin + my_idx];
      const float sy = d.sy[pi.s_begin + my_idx];
      const float sz = d.sz[pi.s_begin + my_idx];
      ex = sx - lx[pos];
      ey = sy - ly[pos];
      ez = sz - lz[pos];
      e2 = ex * ex + ey * ey + ez * ez;
      mx = sy * ez - sz * ey;
      my = sz * ex - sx * ez;
      mz = sx * ey - sy * ex;
      if (d.dbg_rev) d.dbg_rev[(size_t)i * d.mc_max + lm[pos]] = my_idx;
    }
  }
  e2 = wave_sum(e2);
  ex = wave_sum(ex);
  ey = wave_sum(ey);
  ez = wave_sum(ez);
  mx = wave_sum(mx);
  my = wave_sum(my);
  mz = wave_sum(mz);
  if (lane == 0) {
    wpart[w][0] = e2; wpart[w][1] = ex; wpart[w][2] = ey; wpart[w][3] = ez;
    wpart[w][4] = mx; wpart[w][5] = my; wpart[w][6] = mz;
  }
  __syncthreads();
  if (tid < 7) {
    out[tid] = ((wpart[0][tid] + wpart[1][tid]) + wpart[2][tid]) + wpart[3][tid];
  } else if (tid == 7) {
    out[7] = (float)total;
  }
}

void launch_gate_reverse(const Dev& d, hipStream_t s) {
  if (d.total_gate_wgs == 0) return;
  const int grid = ((d.total_gate_wgs + 7) / 8) * 8;
  hipLaunchKernelGGL(k_gate_reverse, dim3(grid), dim3(256), 0, s, d);
}

}  // namespace asicp
