// k_particle.hip -- per-particle completion of an iteration and the final
// selection (Algorithm 1).
//
// k_finalize: sums the partial records in a fixed order, forms the cost
// C = 1/2 (L_ct + lambda L_com) of eqs. (13)-(15) with its translation and
// world rotation-vector gradients (eqs. 16-17 in the 6-D tangent), replaces
// the gradient by the collision gradient of eq. (18) when any point collides,
// and in the SGD-ICP phase applies the convergence test and the update of
// eq. (3).  k_select returns, per object, the lowest-cost collision-free
// particle (Algorithm 1 return).
#include "asicp_internal.h"

namespace asicp {

__device__ __forceinline__ void retract(float t[3], float q[4], const float dt[3], const float dw[3]) {
  t[0] += dt[0];
  t[1] += dt[1];
  t[2] += dt[2];
  const float th = sqrtf(dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2]);
  float ew = 1.f, ex = 0.f, ey = 0.f, ez = 0.f;
  if (th > 0.f) {
    float sh, ch;
    sincosf(0.5f * th, &sh, &ch);
    const float s = sh / th;
    ew = ch; ex = s * dw[0]; ey = s * dw[1]; ez = s * dw[2];
  }
  // (e (x) q)
  const float w = ew * q[0] - ex * q[1] - ey * q[2] - ez * q[3];
  const float x = ew * q[1] + q[0] * ex + (ey * q[3] - ez * q[2]);
  const float y = ew * q[2] + q[0] * ey + (ez * q[1] - ex * q[3]);
  const float z = ew * q[3] + q[0] * ez + (ex * q[2] - ey * q[1]);
  const float nrm = sqrtf(w * w + x * x + y * y + z * z);
  const float sg = (w < 0.f) ? -1.f : 1.f;
  const float inv = sg / nrm;
  q[0] = w * inv; q[1] = x * inv; q[2] = y * inv; q[3] = z * inv;
}

__device__ __forceinline__ bool finite3(float a, float b, float c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// One wavefront per particle: lanes read the partial records in parallel and
// add them with a fixed butterfly; lane 0 finishes the particle.
__global__ __launch_bounds__(256) void k_finalize(Dev d, int k, int final_eval) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= d.Ktot) return;
  const int lane = threadIdx.x & 63;
  const int g = i / d.K;
  const GroupInfo gi = d.groups[g];
  const PreInfo& pi = d.pres[gi.pre];
  const ObjInfo& oi = d.objs[gi.obj];

  // the forward records: one per 16 * 2^qi contact points (one per wave of
  // the forward launch).  Each group of 64 points is completed to the same
  // tree, (b0 + b1) + (b2 + b3) over its blocks of 16, whatever qi is; blocks
  // past the cloud's end count as +0, as they do inside a wave
  float s[7] = {0, 0, 0, 0, 0, 0, 0};
  const float* np = d.nn_part + (size_t)i * d.max_waves_pp * kPartStride;
  const int qi = d.nn_qi, nrec = pi.waves[qi], groups = pi.waves[2];
  for (int c = lane; c < groups; c += 64) {
    if (qi == 2) {
#pragma unroll
      for (int a = 0; a < 7; ++a) s[a] += np[c * kPartStride + a];
    } else if (qi == 1) {
      const bool h = 2 * c + 1 < nrec;
#pragma unroll
      for (int a = 0; a < 7; ++a) {
        const float r0 = np[2 * c * kPartStride + a], r1 = h ? np[(2 * c + 1) * kPartStride + a] : 0.f;
        s[a] += r0 + r1;
      }
    } else {
      float r[4][7];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const bool h = 4 * c + b < nrec;
#pragma unroll
        for (int a = 0; a < 7; ++a) r[b][a] = h ? np[(4 * c + b) * kPartStride + a] : 0.f;
      }
#pragma unroll
      for (int a = 0; a < 7; ++a) s[a] += (r[0][a] + r[1][a]) + (r[2][a] + r[3][a]);
    }
  }
  float cs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const float* cp = d.col_part + (size_t)i * d.max_gate_chunks * kPartStride;
  for (int c = lane; c < oi.gate_chunks; c += 64)
#pragma unroll
    for (int a = 0; a < 8; ++a) cs[a] += cp[c * kPartStride + a];
#pragma unroll
  for (int a = 0; a < 7; ++a) s[a] = wave_sum(s[a]);
#pragma unroll
  for (int a = 0; a < 8; ++a) cs[a] = wave_sum(cs[a]);
  if (lane != 0) return;

  float t[3], q[4], R[9];
  load_pose(d.theta, d.Ktot, i, t, q);
  quat_to_rot(q[0], q[1], q[2], q[3], R);
  const float* pc = d.pre_const + gi.pre * 8;
  const float* com = d.obj_com + gi.obj * 4;
  const float invN = 1.0f / (float)pi.n;
  const float uTx = R[0] * pc[0] + R[1] * pc[1] + R[2] * pc[2];
  const float uTy = R[3] * pc[0] + R[4] * pc[1] + R[5] * pc[2];
  const float uTz = R[6] * pc[0] + R[7] * pc[1] + R[8] * pc[2];
  // the pose relative to the centroid: t and CoM may both be far from the
  // origin, their difference is small
  const float tcx = t[0] - com[0], tcy = t[1] - com[1], tcz = t[2] - com[2];
  const float eTx = uTx + tcx, eTy = uTy + tcy, eTz = uTz + tcz;
  // contact moment: the records hold sum s' x e with s' = R s + (t - CoM)
  s[4] -= tcy * s[3] - tcz * s[2];
  s[5] -= tcz * s[1] - tcx * s[3];
  s[6] -= tcx * s[2] - tcy * s[1];
  const float lam = d.lambda;
  const float cost_ct = 0.5f * (s[0] * invN + lam * (eTx * eTx + eTy * eTy + eTz * eTz));
  float cost_pen = 0.f;
  float gct[6];
  gct[0] = s[1] * invN + lam * eTx;
  gct[1] = s[2] * invN + lam * eTy;
  gct[2] = s[3] * invN + lam * eTz;
  gct[3] = s[4] * invN + lam * (uTy * eTz - uTz * eTy);
  gct[4] = s[5] * invN + lam * (uTz * eTx - uTx * eTz);
  gct[5] = s[6] * invN + lam * (uTx * eTy - uTy * eTx);

  const int ncol = (int)cs[7];
  float gcol[6] = {0, 0, 0, 0, 0, 0}, ccost = 0.f;
  if (ncol > 0) {
    const float inv = 1.0f / (float)ncol;
    const float dx = cs[1] * inv, dy = cs[2] * inv, dz = cs[3] * inv;
    const float mx = cs[4] * inv, my = cs[5] * inv, mz = cs[6] * inv;
    gcol[0] = R[0] * dx + R[1] * dy + R[2] * dz;
    gcol[1] = R[3] * dx + R[4] * dy + R[5] * dz;
    gcol[2] = R[6] * dx + R[7] * dy + R[8] * dz;
    gcol[3] = R[0] * mx + R[1] * my + R[2] * mz;
    gcol[4] = R[3] * mx + R[4] * my + R[5] * mz;
    gcol[5] = R[6] * mx + R[7] * my + R[8] * mz;
    ccost = 0.5f * cs[0] * inv;
  }
  if (d.w_pen > 0.f && oi.mc > 0) {  // optional penetration term, added to C and its gradient
    float pn[7] = {0, 0, 0, 0, 0, 0, 0};
    const float* pp = d.pen_part + (size_t)i * d.max_gate_chunks * kPartStride;
    for (int c = 0; c < oi.gate_chunks; ++c)
      for (int a = 0; a < 7; ++a) pn[a] += pp[c * kPartStride + a];
    const float sw = d.w_pen / (float)oi.mc;
    cost_pen = sw * pn[0];
    gct[0] += sw * (R[0] * pn[1] + R[1] * pn[2] + R[2] * pn[3]);
    gct[1] += sw * (R[3] * pn[1] + R[4] * pn[2] + R[5] * pn[3]);
    gct[2] += sw * (R[6] * pn[1] + R[7] * pn[2] + R[8] * pn[3]);
    gct[3] += sw * (R[0] * pn[4] + R[1] * pn[5] + R[2] * pn[6]);
    gct[4] += sw * (R[3] * pn[4] + R[4] * pn[5] + R[5] * pn[6]);
    gct[5] += sw * (R[6] * pn[4] + R[7] * pn[5] + R[8] * pn[6]);
  }
  const float cost = cost_ct + cost_pen;
  const float* gf = ncol > 0 ? gcol : gct;
  const int K = d.Ktot;
  d.cost[i] = cost;
  d.col_cost[i] = ccost;
  d.ncol[i] = ncol;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    d.grad[a * K + i] = gf[a];
    d.grad_ct[a * K + i] = gct[a];
    d.grad_col[a * K + i] = gcol[a];
  }
  bool ok = isfinite(cost) && isfinite(ccost) && finite3(gf[0], gf[1], gf[2]) &&
            finite3(gf[3], gf[4], gf[5]) && finite3(t[0], t[1], t[2]) &&
            finite3(q[0], q[1], q[2]) && isfinite(q[3]);
  if (!ok) atomicOr(d.flags, 1);
  if (final_eval) return;

  int conv = d.converged[i];
  if (ncol > 0) conv = 0;
  if (k >= d.k_stein) {
    const float prev = d.prev_cost[i];
    if (!conv && ncol == 0 && prev > 0.f && fabsf(cost - prev) < d.conv_tol * prev) conv = 1;
    const float at = pc[4], aw = pc[5];
    float dt[3] = {-at * gf[0], -at * gf[1], -at * gf[2]};
    float dw[3] = {-aw * gf[3], -aw * gf[4], -aw * gf[5]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d.phi[a * K + i] = conv ? 0.f : dt[a];
      d.phi[(3 + a) * K + i] = conv ? 0.f : dw[a];
    }
    if (!conv) {
      const float e = d.eta;
      const float sdt[3] = {e * dt[0], e * dt[1], e * dt[2]};
      const float sdw[3] = {e * dw[0], e * dw[1], e * dw[2]};
      retract(t, q, sdt, sdw);
      d.theta[0 * K + i] = t[0];
      d.theta[1 * K + i] = t[1];
      d.theta[2 * K + i] = t[2];
      d.theta[3 * K + i] = q[0];
      d.theta[4 * K + i] = q[1];
      d.theta[5 * K + i] = q[2];
      d.theta[6 * K + i] = q[3];
    }
  }
  d.converged[i] = conv;
  d.prev_cost[i] = cost;
}

// lexicographic key: collision-free first, then cost (NaN as +inf), then index
__device__ __forceinline__ bool better(int fa, float ca, int ia, int fb, float cb, int ib) {
  if (fa != fb) return fa > fb;
  if (ca != cb) return ca < cb;
  return ia < ib;
}

__global__ __launch_bounds__(256) void k_select(Dev d) {
  __shared__ int sf[256], si[256];
  __shared__ float sc[256];
  const int o = blockIdx.x, tid = threadIdx.x;
  const int per = d.n_pre * d.K, base = o * per;
  int bf = -1, bi = 0x7fffffff;
  float bc = __builtin_inff();
  for (int i = base + tid; i < base + per; i += 256) {
    float c = d.cost[i];
    if (!(c == c)) c = __builtin_inff();
    const int f = d.ncol[i] == 0;
    if (bf < 0 || better(f, c, i, bf, bc, bi)) { bf = f; bc = c; bi = i; }
  }
  sf[tid] = bf; sc[tid] = bc; si[tid] = bi;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (tid < off) {
      const int f2 = sf[tid + off];
      if (f2 >= 0 && (sf[tid] < 0 || better(f2, sc[tid + off], si[tid + off], sf[tid], sc[tid], si[tid]))) {
        sf[tid] = f2; sc[tid] = sc[tid + off]; si[tid] = si[tid + off];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const int b = si[0];
    d.best[2 * o] = b;
    d.best[2 * o + 1] = sf[0];
    for (int a = 0; a < 7; ++a) d.best_theta[8 * o + a] = d.theta[a * d.Ktot + b];
    d.best_theta[8 * o + 7] = d.cost[b];
  }
}

void launch_finalize(const Dev& d, int k, int final_eval, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3((d.Ktot + 3) / 4), dim3(256), 0, s, d, k, final_eval);
}

void launch_select(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(d.n_obj), dim3(256), 0, s, d);
}

}  // namespace asicp
