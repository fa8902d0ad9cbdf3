// k_gate_reverse.hip -- SDF collision gate and reverse nearest neighbour
// (Sec. IV-C and eq. (18); Algorithm 1's collision branch).
//
// One workgroup = one particle x 2048 points of its collision cloud.  Each
// point is moved into the gripper frame, c' = R^T (c - t), and looked up in
// the preshape's SDF by trilinear interpolation; it collides when it lies in
// the node box and the value is strictly negative.  Colliding points are
// compacted in the cloud's order and paired with their nearest contact point in
// the gripper frame (a rigid motion preserves distances, so this is the
// nearest transformed contact point of eq. (18)).  Partial sums, gripper
// frame: [sum |s - c'|^2, sum (s - c') (3), sum s x (s - c') (3), count].
//
// Trilinear weights are non-negative, so a point can only collide inside a
// cell with a negative corner.  Without reading the grid, whole workgroups
// (the transformed box of the workgroup's own 2048 points, compact because
// the cloud is in k-d leaf order) and 64-point leaves are culled by the box
// of negative nodes and the brick counts of the set-up's SDF tables, and
// single points by their cell's bit.  Every test is exact.  A workgroup finds
// its particle and chunk in the set-up's table of gate workgroups.
#include "nn_core.h"

namespace asicp {

constexpr int kPerThread = kGateChunk / 256;
constexpr int kGateBatch = 4;  // points whose SDF node values are in flight together
#ifndef ASICP_REV_Q
#define ASICP_REV_Q 2
#endif
constexpr int kRevQ = ASICP_REV_Q;  // blocks of 16 colliding points per reverse scan (1, 2 or 4)

// Workgroup placement over the XCDs, as for the forward kernel (MAP 0:
// contiguous work per XCD, MAP 1: dispatch order); changes no result.
template <int MAP>
__device__ __forceinline__ int xcd_logical_g(int b, int nwg) {
  if (MAP == 1) return b;
  const int per = (nwg + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

// Cell of a gripper-frame point for the trilinear SDF: false if the point
// lies outside the node box or in a cell without a negative corner (it cannot
// collide); otherwise off = index of the cell's lowest node and f = the
// point's fractions within the cell.  No memory is read.
__device__ __forceinline__ bool sdf_cell(const PreInfo& pi, float px, float py, float pz, int& off,
                                         float f[3]) {
  const float ux = (px - pi.ox) * pi.inv_cell;
  const float uy = (py - pi.oy) * pi.inv_cell;
  const float uz = (pz - pi.oz) * pi.inv_cell;
  if (!(ux >= 0.f && ux <= (float)(pi.nx - 1) && uy >= 0.f && uy <= (float)(pi.ny - 1) &&
        uz >= 0.f && uz <= (float)(pi.nz - 1)))
    return false;
  const int ix = min((int)floorf(ux), pi.nx - 2);
  const int iy = min((int)floorf(uy), pi.ny - 2);
  const int iz = min((int)floorf(uz), pi.nz - 2);
  if (ix < pi.neg_lo[0] - 1 || ix > pi.neg_hi[0] || iy < pi.neg_lo[1] - 1 || iy > pi.neg_hi[1] ||
      iz < pi.neg_lo[2] - 1 || iz > pi.neg_hi[2])
    return false;
  if (!((pi.cell_bits[((long long)iz * (pi.ny - 1) + iy) * pi.cbw + (ix >> 5)] >> (ix & 31)) & 1u)) return false;
  f[0] = ux - (float)ix;
  f[1] = uy - (float)iy;
  f[2] = uz - (float)iz;
  off = (iz * pi.ny + iy) * pi.nx + ix;
  return true;
}

// The cell's 8 node values, v[4 dz + 2 dy + dx].
__device__ __forceinline__ void sdf_corners(const PreInfo& pi, int off, float v[8]) {
  const int sy = pi.nx, sz = pi.nx * pi.ny;
  const float* g = pi.sdf + off;
  v[0] = g[0]; v[1] = g[1]; v[2] = g[sy]; v[3] = g[sy + 1];
  v[4] = g[sz]; v[5] = g[sz + 1]; v[6] = g[sz + sy]; v[7] = g[sz + sy + 1];
}

// Trilinear value at fractions f from the cell's node values, and, if grad is
// given, the interpolant's gradient (world units).
__device__ __forceinline__ float sdf_interp(const float v[8], const float f[3], float inv_cell, float* grad) {
  const float fx = f[0], fy = f[1], fz = f[2];
  const float v000 = v[0], v100 = v[1], v010 = v[2], v110 = v[3];
  const float v001 = v[4], v101 = v[5], v011 = v[6], v111 = v[7];
  const float c00 = (1.f - fx) * v000 + fx * v100;
  const float c10 = (1.f - fx) * v010 + fx * v110;
  const float c01 = (1.f - fx) * v001 + fx * v101;
  const float c11 = (1.f - fx) * v011 + fx * v111;
  const float c0 = (1.f - fy) * c00 + fy * c10;
  const float c1 = (1.f - fy) * c01 + fy * c11;
  const float val = (1.f - fz) * c0 + fz * c1;
  if (grad) {
    const float gx = (1.f - fy) * (1.f - fz) * (v100 - v000) + fy * (1.f - fz) * (v110 - v010) +
                     (1.f - fy) * fz * (v101 - v001) + fy * fz * (v111 - v011);
    const float gy = (1.f - fx) * (1.f - fz) * (v010 - v000) + fx * (1.f - fz) * (v110 - v100) +
                     (1.f - fx) * fz * (v011 - v001) + fx * fz * (v111 - v101);
    grad[0] = gx * inv_cell;
    grad[1] = gy * inv_cell;
    grad[2] = (c1 - c0) * inv_cell;
  }
  return val;
}

// Can any point of a box of collision points (lo = bx[0..2], hi = bx[4..6])
// reach a cell with a negative node?  The box is moved into the gripper frame
// as centre R^T (c - t) and half extents |R^T| e (the box of its rotated
// corners), widened by 10 um for the rounding of the per-point transform; it
// must meet the box of cells next to negative nodes, and the bricks its cells
// fall in must hold such a cell (8 entries of the brick counts).  A point's
// cell index is a monotone function of its coordinate, so the cells of the
// points lie in the range computed from the box's bounds.  An empty box
// (lo > hi) never collides.
__device__ __forceinline__ bool box_may_collide(const PreInfo& pi, const float* bx, const float R[9],
                                                const float t[3]) {
  if (pi.neg_hi[0] < 0) return false;  // no negative node at all
  if (!(bx[0] <= bx[4] && bx[1] <= bx[5] && bx[2] <= bx[6])) return false;
  const float cx = 0.5f * (bx[0] + bx[4]) - t[0], cy = 0.5f * (bx[1] + bx[5]) - t[1],
              cz = 0.5f * (bx[2] + bx[6]) - t[2];
  const float ex = 0.5f * (bx[4] - bx[0]), ey = 0.5f * (bx[5] - bx[1]), ez = 0.5f * (bx[6] - bx[2]);
  const float c[3] = {R[0] * cx + R[3] * cy + R[6] * cz, R[1] * cx + R[4] * cy + R[7] * cz,
                      R[2] * cx + R[5] * cy + R[8] * cz};
  const float e[3] = {fabsf(R[0]) * ex + fabsf(R[3]) * ey + fabsf(R[6]) * ez,
                      fabsf(R[1]) * ex + fabsf(R[4]) * ey + fabsf(R[7]) * ez,
                      fabsf(R[2]) * ex + fabsf(R[5]) * ey + fabsf(R[8]) * ez};
  const float o[3] = {pi.ox, pi.oy, pi.oz};
  const int n[3] = {pi.nx, pi.ny, pi.nz};
  const float margin = 1e-5f;
  int b0[3], b1[3];
  for (int a = 0; a < 3; ++a) {
    const float lo = c[a] - e[a] - margin, hi = c[a] + e[a] + margin;
    const float g0 = o[a] + (float)(pi.neg_lo[a] - 1) * pi.cell - margin;
    const float g1 = o[a] + (float)(pi.neg_hi[a] + 1) * pi.cell + margin;
    if (!(hi >= g0 && lo <= g1)) return false;
    // cells of the points, as the per-point lookup computes them (outside
    // the node box no point collides)
    const float u0 = (lo - o[a]) * pi.inv_cell, u1 = (hi - o[a]) * pi.inv_cell;
    if (!(u1 >= 0.f && u0 <= (float)(n[a] - 1))) return false;
    const int i0 = u0 > 0.f ? (int)fminf(floorf(u0), (float)(n[a] - 2)) : 0;
    const int i1 = (int)fminf(floorf(u1), (float)(n[a] - 2));
    b0[a] = i0 / kBrick;
    b1[a] = i1 / kBrick + 1;
  }
  const long long ex1 = pi.bnx + 1, pl = ex1 * (pi.bny + 1);
  auto at = [&](int x, int y, int z) { return pi.brick_sum[(long long)z * pl + (long long)y * ex1 + x]; };
  const int cnt = (at(b1[0], b1[1], b1[2]) - at(b0[0], b1[1], b1[2]) - at(b1[0], b0[1], b1[2]) -
                   at(b1[0], b1[1], b0[2])) +
                  (at(b0[0], b0[1], b1[2]) + at(b0[0], b1[1], b0[2]) + at(b1[0], b0[1], b0[2]) -
                   at(b0[0], b0[1], b0[2]));
  return cnt > 0;
}

// Reverse NN of Q blocks of colliding points (gripper frame) against the
// k-d ordered contact cloud, skipping contact chunks that cannot hold a
// nearest point (same exact result as scanning them all).
template <int Q>
__device__ __forceinline__ void rev_scan(const Dev& d, const PreInfo& pi, int gi_pre, const float* bq, int* idx) {
  const int lane = threadIdx.x & 63;
  float snorm[Q];
  int vq[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    // the lane's query: components from the four rows at its position
    const float x = __shfl(bq[q], (lane & 15), 64);
    const float y = __shfl(bq[q], (lane & 15) + 16, 64);
    const float z = __shfl(bq[q], (lane & 15) + 32, 64);
    snorm[q] = x * x + y * y + z * z;
    vq[q] = 16;
  }
  nn_scan_pruned<Q, false, false, kChunkTG>(d.pre_prep + (size_t)pi.prep_tg_begin * 64, pi.ntg, pi.n,
                                  d.pre_box + (size_t)pi.prep_tg_begin / kChunkTG * 8, nullptr, bq, snorm, nullptr, vq,
                                  d.pre_const[8 * gi_pre + 6], idx, d.flags + 1);
}

template <int MAP>
__global__ __launch_bounds__(256) void k_gate_reverse(Dev d) {
  __shared__ float lx[kGateChunk], ly[kGateChunk], lz[kGateChunk];
  __shared__ int lm[kGateChunk];
  __shared__ int wcnt[kPerThread][4];
  __shared__ float wpart[4][kPartStride];

  const int nwg = d.total_gate_wgs;
  const int logical = xcd_logical_g<MAP>(blockIdx.x, nwg);
  if (logical >= nwg) return;  // uniform over the workgroup
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;

  const GateWG gw = d.gate_wg[logical];
  const GroupInfo gi = d.groups[gw.g];
  const PreInfo& pi = d.pres[gi.pre];
  const ObjInfo& oi = d.objs[gi.obj];
  const int cc = gw.cc, i = gw.i;
  float* out = d.col_part + ((size_t)i * d.max_gate_chunks + cc) * kPartStride;

  // the pose relative to the object's centroid, like the stored collision
  // cloud: c' = R^T ((c - com) - (t - com))
  float t[3], qv[4], R[9];
  load_pose(d.theta, d.Ktot, i, t, qv);
  quat_to_rot(qv[0], qv[1], qv[2], qv[3], R);
  {
    const float* com = d.obj_com + 4 * gi.obj;
    for (int a = 0; a < 3; ++a) t[a] = uniform_f(t[a] - com[a]);
  }

  float* pout = d.pen_part + ((size_t)i * d.max_gate_chunks + cc) * kPartStride;
  // the box of this workgroup's 2048 points (spatially compact: the cloud is
  // k-d ordered), not of the whole cloud, so most far chunks stop here
  if (!box_may_collide(pi, d.col_box + (size_t)gw.box * 8, R, t)) {
    if (tid < kPartStride) {
      out[tid] = 0.f;
      pout[tid] = 0.f;
    }
    if (d.dbg_rev)
      for (int r = 0; r < kPerThread; ++r) {
        const int m = cc * kGateChunk + r * 256 + tid;
        if (m < oi.mc) d.dbg_rev[(size_t)i * d.mc_max + d.col_perm[oi.c_begin + m]] = -1;
      }
    return;
  }

  // gate: thread tid owns points cc*2048 + r*256 + tid, r = 0..7, of the
  // k-d ordered collision cloud (so colliding points come out clustered).
  // In round r the wave's 64 points are one 64-point leaf (r * 4 + w of the
  // chunk); lane r tests that leaf's box, and rounds whose leaf cannot reach
  // a negative cell load no point (bit r of lmask, uniform over the wave)
  unsigned int lmask;
  {
    bool ok = false;
    if (lane < kPerThread)
      ok = box_may_collide(pi, d.col_leaf_box + (((size_t)oi.gbox_begin + cc) * (kGateChunk / 64) + lane * 4 + w) * 8,
                            R, t);
    lmask = (unsigned int)__ballot(ok);
  }
  unsigned int bits = 0u;
  float px[kPerThread], py[kPerThread], pz[kPerThread];
  // penetration sums (gripper frame): phi^2, -2 phi grad, 2 phi grad x c'
  float pn[7] = {0, 0, 0, 0, 0, 0, 0};
  const bool want_pen = d.w_pen > 0.f;
  // all eight points are loaded and moved first, and the node values of a
  // batch of kGateBatch points are requested together before any is used,
  // so their memory latencies overlap
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    px[r] = py[r] = pz[r] = 0.f;
    if (!((lmask >> r) & 1u)) continue;
    const int m = cc * kGateChunk + r * 256 + tid;
    const float4 c = d.col_pts[oi.c_begin + max(0, min(m, oi.mc - 1))];
    const float dx = c.x - t[0];
    const float dy = c.y - t[1];
    const float dz = c.z - t[2];
    px[r] = R[0] * dx + R[3] * dy + R[6] * dz;
    py[r] = R[1] * dx + R[4] * dy + R[7] * dz;
    pz[r] = R[2] * dx + R[5] * dy + R[8] * dz;
  }
#pragma unroll
  for (int r0 = 0; r0 < kPerThread; r0 += kGateBatch) {
    bool cand[kGateBatch];
    int off[kGateBatch];
    float fr[kGateBatch][3], v[kGateBatch][8];
#pragma unroll
    for (int u = 0; u < kGateBatch; ++u) {
      const int r = r0 + u;
      off[u] = 0;
      cand[u] = ((lmask >> r) & 1u) && cc * kGateChunk + r * 256 + tid < oi.mc &&
                sdf_cell(pi, px[r], py[r], pz[r], off[u], fr[u]);
      if (cand[u]) sdf_corners(pi, off[u], v[u]);
    }
#pragma unroll
    for (int u = 0; u < kGateBatch; ++u) {
      const int r = r0 + u;
      const int m = cc * kGateChunk + r * 256 + tid;
      if (m >= oi.mc) continue;
      float phi = 0.f, gr[3];
      const bool col = cand[u] && (phi = sdf_interp(v[u], fr[u], pi.inv_cell, want_pen ? gr : nullptr)) < 0.f;
      if (col && want_pen) {
        pn[0] += phi * phi;
        pn[1] -= 2.f * phi * gr[0];
        pn[2] -= 2.f * phi * gr[1];
        pn[3] -= 2.f * phi * gr[2];
        pn[4] += 2.f * phi * (gr[1] * pz[r] - gr[2] * py[r]);
        pn[5] += 2.f * phi * (gr[2] * px[r] - gr[0] * pz[r]);
        pn[6] += 2.f * phi * (gr[0] * py[r] - gr[1] * px[r]);
      }
      if (col) bits |= 1u << r;
      else if (d.dbg_rev) d.dbg_rev[(size_t)i * d.mc_max + d.col_perm[oi.c_begin + m]] = -1;
    }
  }
  // compaction in the cloud's (k-d) order, point m = cc*2048 + r*256 + tid:
  // slot r's ballot ranks the lane within its wave, and the per-slot wave
  // counts place the wave, so a block of 16 consecutive colliding points is
  // spatially compact and the reverse scan's chunk bounds stay tight
  int rank[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    const unsigned long long bal = __ballot((bits >> r) & 1u);
    rank[r] = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0u));
    if (lane == 0) wcnt[r][w] = __popcll(bal);
  }
  __syncthreads();
  int total = 0;
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    int before = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) before += (k < w) ? wcnt[r][k] : 0;
    rank[r] += total + before;
    total += (wcnt[r][0] + wcnt[r][1]) + (wcnt[r][2] + wcnt[r][3]);
  }
  if (want_pen) {  // fixed-order workgroup sums of the penetration terms
#pragma unroll
    for (int a = 0; a < 7; ++a) pn[a] = wave_sum(pn[a]);
    if (lane == 0)
      for (int a = 0; a < 7; ++a) wpart[w][a] = pn[a];
    __syncthreads();
    if (tid < 7) pout[tid] = ((wpart[0][tid] + wpart[1][tid]) + wpart[2][tid]) + wpart[3][tid];
    __syncthreads();
  } else if (tid < kPartStride) {
    pout[tid] = 0.f;
  }
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    if (bits & (1u << r)) {
      const int pos = rank[r];
      lx[pos] = px[r]; ly[pos] = py[r]; lz[pos] = pz[r];
      lm[pos] = cc * kGateChunk + r * 256 + tid;
    }
  }
  __syncthreads();
  if (total == 0) {
    if (tid < kPartStride) out[tid] = 0.f;
    return;
  }
  // reverse NN: blocks of 16 colliding points; wave w takes blocks w, w+4, ...
  // in batches of up to kRevQ blocks per scan of the contact cloud (few
  // blocks per scan keep the kernel's registers within what one retiring
  // forward-NN workgroup frees, so it can run beside that launch)
  const int nb = (total + 15) >> 4;
  const int nbw = (nb > w) ? (nb - w + 3) >> 2 : 0;
  const int comp = lane >> 4;
  float e2 = 0.f, ex = 0.f, ey = 0.f, ez = 0.f, mx = 0.f, my = 0.f, mz = 0.f;
  for (int k0 = 0; k0 < nbw; k0 += kRevQ) {
    const int qn = min(kRevQ, nbw - k0);
    float bq[kRevQ];
    const int pfirst = (w + 4 * k0) * 16;  // a colliding point of this batch
#pragma unroll
    for (int q = 0; q < kRevQ; ++q) {
      int p = (w + 4 * (k0 + q)) * 16 + (lane & 15);
      if (!(q < qn && p < total)) p = pfirst;  // padding queries repeat it
      const float v = comp == 0 ? lx[p] : comp == 1 ? ly[p] : lz[p];
      bq[q] = comp == 3 ? 1.0f : v;
    }
    int idx[kRevQ];
#pragma unroll
    for (int q = 0; q < kRevQ; ++q) idx[q] = 0;
    if (kRevQ == 1 || qn == 1) rev_scan<1>(d, pi, gi.pre, bq, idx);
    else rev_scan<kRevQ>(d, pi, gi.pre, bq, idx);
    int my_idx = idx[0];
#pragma unroll
    for (int q = 1; q < kRevQ; ++q)
      if (comp == q) my_idx = idx[q];
    const int p = (w + 4 * (k0 + comp)) * 16 + (lane & 15);
    if (comp < qn && p < total) {
      if (my_idx >= pi.n) {
        atomicOr(d.flags + 1, 4);
        my_idx = pi.n - 1;
      }
      const float4 sp = d.pre_pts[(size_t)pi.prep_tg_begin * 64 + my_idx];  // k-d ordered copy
      const float sx = sp.x, sy = sp.y, sz = sp.z;
      const float dx = sx - lx[p], dy = sy - ly[p], dz = sz - lz[p];
      e2 += dx * dx + dy * dy + dz * dz;
      ex += dx; ey += dy; ez += dz;
      mx += sy * dz - sz * dy;
      my += sz * dx - sx * dz;
      mz += sx * dy - sy * dx;
      if (d.dbg_rev)
        d.dbg_rev[(size_t)i * d.mc_max + d.col_perm[oi.c_begin + lm[p]]] =
            d.pre_perm[(size_t)pi.prep_tg_begin * 64 + my_idx];
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
  if (d.xcd_map) hipLaunchKernelGGL(k_gate_reverse<1>, dim3(grid), dim3(256), 0, s, d);
  else hipLaunchKernelGGL(k_gate_reverse<0>, dim3(grid), dim3(256), 0, s, d);
}

}  // namespace asicp
