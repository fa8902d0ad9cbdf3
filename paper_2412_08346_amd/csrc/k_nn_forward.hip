// k_nn_forward.hip -- transform, forward nearest neighbour and contact-loss
// partial sums (Algorithm 1: transform the source cloud, pair it with the
// object cloud by eq. (1), accumulate the terms of eqs. (14), (16), (17)).
//
// One wavefront = one particle x 64 contact points, matched against the whole
// object cloud of its group with the MFMA core.  Partial sums per wavefront:
// [sum |e|^2, sum e (3), sum (R s) x e (3), points], e = s' - r_nn.
#include "nn_core.h"

namespace asicp {

// Hardware places workgroup b on XCD b % 8; give each XCD a contiguous range
// of logical workgroups so that one XCD's L2 serves the same objects.
__device__ __forceinline__ int xcd_logical(int b, int nwg) {
  const int per = (nwg + 7) >> 3;
  return (b & 7) * per + (b >> 3);
}

__global__ __launch_bounds__(256) void k_nn_forward(Dev d) {
  const int nwg = (d.total_waves + 3) >> 2;
  const int logical = xcd_logical(blockIdx.x, nwg);
  if (logical >= nwg) return;
  const int wave = logical * 4 + (threadIdx.x >> 6);
  if (wave >= d.total_waves) return;
  const int lane = threadIdx.x & 63;

  int lo = 0, hi = d.G - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.groups[mid].wave_off <= wave) lo = mid; else hi = mid - 1;
  }
  const GroupInfo gi = d.groups[lo];
  const PreInfo& pi = d.pres[gi.pre];
  const ObjInfo& oi = d.objs[gi.obj];
  const int local = wave - gi.wave_off;
  const int pj = local / pi.waves, chunk = local - pj * pi.waves;
  const int i = lo * d.K + pj;

  float t[3], qv[4], R[9];
  load_pose(d.theta, d.Ktot, i, t, qv);
  quat_to_rot(qv[0], qv[1], qv[2], qv[3], R);

  const int comp = lane >> 4;
  float bq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int n = chunk * 64 + q * 16 + (lane & 15);
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if (n < pi.n) {
      sx = d.sx[pi.s_begin + n];
      sy = d.sy[pi.s_begin + n];
      sz = d.sz[pi.s_begin + n];
    }
    const float px = R[0] * sx + R[1] * sy + R[2] * sz + t[0];
    const float py = R[3] * sx + R[4] * sy + R[5] * sz + t[1];
    const float pz = R[6] * sx + R[7] * sy + R[8] * sz + t[2];
    bq[q] = comp == 0 ? px : comp == 1 ? py : comp == 2 ? pz : 1.0f;
  }
  int idx[4];
  nn_scan<4>(d.obj_prep + (size_t)oi.prep_tg_begin * 64, oi.ntg, bq, idx, d.flags + 1);

  // lane l now owns contact point chunk*64 + l (block l/16, query l%16)
  int my = idx[0];
  if (comp == 1) my = idx[1];
  if (comp == 2) my = idx[2];
  if (comp == 3) my = idx[3];
  const int n = chunk * 64 + lane;
  float e2 = 0.f, ex = 0.f, ey = 0.f, ez = 0.f, mx = 0.f, my_ = 0.f, mz = 0.f, cnt = 0.f;
  if (n < pi.n) {
    if (my >= oi.m) {
      atomicOr(d.flags + 1, 2);
      my = oi.m - 1;
    }
    const float sx = d.sx[pi.s_begin + n], sy = d.sy[pi.s_begin + n], sz = d.sz[pi.s_begin + n];
    const float ux = R[0] * sx + R[1] * sy + R[2] * sz;
    const float uy = R[3] * sx + R[4] * sy + R[5] * sz;
    const float uz = R[6] * sx + R[7] * sy + R[8] * sz;
    ex = ux + t[0] - d.rx[oi.r_begin + my];
    ey = uy + t[1] - d.ry[oi.r_begin + my];
    ez = uz + t[2] - d.rz[oi.r_begin + my];
    e2 = ex * ex + ey * ey + ez * ez;
    mx = uy * ez - uz * ey;
    my_ = uz * ex - ux * ez;
    mz = ux * ey - uy * ex;
    cnt = 1.f;
    if (d.dbg_nn) d.dbg_nn[(size_t)i * d.n_max + n] = my;
  }
  e2 = wave_sum(e2);
  ex = wave_sum(ex);
  ey = wave_sum(ey);
  ez = wave_sum(ez);
  mx = wave_sum(mx);
  my_ = wave_sum(my_);
  mz = wave_sum(mz);
  cnt = wave_sum(cnt);
  if (lane == 0) {
    float* out = d.nn_part + ((size_t)i * d.max_waves_pp + chunk) * kPartStride;
    out[0] = e2; out[1] = ex; out[2] = ey; out[3] = ez;
    out[4] = mx; out[5] = my_; out[6] = mz; out[7] = cnt;
  }
}

void launch_nn_forward(const Dev& d, hipStream_t s) {
  const int nwg = (d.total_waves + 3) / 4;
  const int grid = ((nwg + 7) / 8) * 8;
  hipLaunchKernelGGL(k_nn_forward, dim3(grid), dim3(256), 0, s, d);
}

}  // namespace asicp
