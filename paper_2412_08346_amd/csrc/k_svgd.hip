// k_svgd.hip -- annealed Stein ICP update of one group (eqs. (6)-(11)).
//
// One workgroup per (object, preshape) group of K <= 1024 particles, all in
// LDS.  (1) bandwidth h of the RBF kernel (eq. 9): lower median of the
// squared translation distances over pairs, by a 4-pass radix select on the
// FP32 bit patterns (monotone for non-negative floats), divided by ln K and
// floored; (2) Stein direction in the 6-D tangent: kernel-weighted mean of
// the preconditioned driving terms -gamma A g_j plus tau times the kernel
// gradient with respect to particle j (translation part scaled by h/2);
// (3) pose update t += eta phi_t, q <- canon(normalize(Exp(eta phi_w) (x) q)).
// All phi are computed from the poses of the same iteration before any pose
// is written back.
#include "asicp_internal.h"

namespace asicp {

constexpr int kMaxK = 1024;

__device__ __forceinline__ float d2_pair(const float* st, int i, int j) {
  const float dx = st[3 * i + 0] - st[3 * j + 0];
  const float dy = st[3 * i + 1] - st[3 * j + 1];
  const float dz = st[3 * i + 2] - st[3 * j + 2];
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

__global__ __launch_bounds__(256) void k_svgd(Dev d, float gamma, float tau, float inv_log_k) {
  __shared__ float st[kMaxK * 3];
  __shared__ float sq[kMaxK * 4];
  __shared__ float sg[kMaxK * 6];
  __shared__ unsigned int hist[256];
  __shared__ unsigned int s_prefix, s_mask, s_rank;
  __shared__ float s_h;

  const int g = blockIdx.x, tid = threadIdx.x, K = d.K, Kt = d.Ktot;
  const int base = g * K;
  for (int j = tid; j < K; j += 256) {
    const int i = base + j;
    for (int a = 0; a < 3; ++a) st[3 * j + a] = d.theta[a * Kt + i];
    for (int a = 0; a < 4; ++a) sq[4 * j + a] = d.theta[(3 + a) * Kt + i];
    for (int a = 0; a < 6; ++a) sg[6 * j + a] = d.grad[a * Kt + i];
  }
  if (tid == 0) {
    s_prefix = 0u;
    s_mask = 0u;
    const unsigned int P = (unsigned int)K * (unsigned int)(K - 1) / 2u;
    s_rank = (K >= 2) ? 2u * ((P - 1u) / 2u) : 0u;  // rank in the doubled (i != j) multiset
  }
  __syncthreads();

  float h;
  if (d.bw_mode == ASICP_BW_FIXED) {
    h = d.h_fixed;
  } else if (K < 2) {
    h = 1.0f;
  } else {
    for (int pass = 0; pass < 4; ++pass) {
      const int shift = 24 - 8 * pass;
      hist[tid] = 0u;
      __syncthreads();
      const unsigned int prefix = s_prefix, mask = s_mask;
      for (int i = tid; i < K; i += 256)
        for (int j = 0; j < K; ++j) {
          if (j == i) continue;
          const unsigned int bits = __float_as_uint(d2_pair(st, i, j));
          if ((bits & mask) == prefix) atomicAdd(&hist[(bits >> shift) & 255u], 1u);
        }
      __syncthreads();
      if (tid == 0) {
        unsigned int cum = 0u, r = s_rank;
        for (int b = 0; b < 256; ++b) {
          if (cum + hist[b] > r) {
            s_prefix = prefix | ((unsigned int)b << shift);
            s_mask = mask | (255u << shift);
            s_rank = r - cum;
            break;
          }
          cum += hist[b];
        }
      }
      __syncthreads();
    }
    const float med = __uint_as_float(s_prefix);
    h = fmaxf(med * inv_log_k, d.h_min);
  }
  if (tid == 0) {
    s_h = h;
    d.h[g] = h;
  }
  __syncthreads();
  h = s_h;
  const float inv_h = 1.0f / h;

  const GroupInfo gi = d.groups[g];
  const float at = d.pre_const[gi.pre * 8 + 4], aw = d.pre_const[gi.pre * 8 + 5];
  const float ga_t = gamma * at, ga_w = gamma * aw;
  const bool block = d.kernel_mode == ASICP_KERNEL_BLOCK;
  const float invK = 1.0f / (float)K;
  float newv[4][7];
  int cnt = 0;
  for (int ii = tid; ii < K; ii += 256, ++cnt) {
    const float tix = st[3 * ii], tiy = st[3 * ii + 1], tiz = st[3 * ii + 2];
    const float qw = sq[4 * ii], qx = sq[4 * ii + 1], qy = sq[4 * ii + 2], qz = sq[4 * ii + 3];
    float acc[6] = {0, 0, 0, 0, 0, 0};
    for (int j = 0; j < K; ++j) {
      const float dx = tix - st[3 * j], dy = tiy - st[3 * j + 1], dz = tiz - st[3 * j + 2];
      const float kt = expf(-__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)) * inv_h);
      const float pw = sq[4 * j], px = sq[4 * j + 1], py = sq[4 * j + 2], pz = sq[4 * j + 3];
      const float dot = qw * pw + qx * px + qy * py + qz * pz;
      const float kr = fabsf(dot);
      const float sgn = dot >= 0.f ? 1.f : -1.f;
      float wdt, wrt, wdw, wrw;
      if (block) {
        wdt = kt; wrt = kt; wdw = kr; wrw = sgn;
      } else {
        wdt = kt * kr; wrt = wdt; wdw = wdt; wrw = kt * sgn;
      }
      // vector part of q_i (x) conj(q_j)
      const float vx = -qw * px + pw * qx + (qy * (-pz) - qz * (-py));
      const float vy = -qw * py + pw * qy + (qz * (-px) - qx * (-pz));
      const float vz = -qw * pz + pw * qz + (qx * (-py) - qy * (-px));
      const float* gj = sg + 6 * j;
      acc[0] += wdt * (-ga_t * gj[0]) + tau * wrt * dx;
      acc[1] += wdt * (-ga_t * gj[1]) + tau * wrt * dy;
      acc[2] += wdt * (-ga_t * gj[2]) + tau * wrt * dz;
      acc[3] += wdw * (-ga_w * gj[3]) + tau * wrw * 0.5f * vx;
      acc[4] += wdw * (-ga_w * gj[4]) + tau * wrw * 0.5f * vy;
      acc[5] += wdw * (-ga_w * gj[5]) + tau * wrw * 0.5f * vz;
    }
    const int i = base + ii;
    float phi[6];
    for (int a = 0; a < 6; ++a) {
      phi[a] = acc[a] * invK;
      d.phi[a * Kt + i] = phi[a];
    }
    // t += eta phi_t ; q <- canon(normalize(Exp(eta phi_w) (x) q))
    const float e = d.eta;
    const float wx = e * phi[3], wy = e * phi[4], wz = e * phi[5];
    const float th = sqrtf(wx * wx + wy * wy + wz * wz);
    float ew = 1.f, ex = 0.f, ey = 0.f, ez = 0.f;
    if (th > 0.f) {
      float sh, ch;
      sincosf(0.5f * th, &sh, &ch);
      const float s = sh / th;
      ew = ch; ex = s * wx; ey = s * wy; ez = s * wz;
    }
    const float nw = ew * qw - ex * qx - ey * qy - ez * qz;
    const float nx = ew * qx + qw * ex + (ey * qz - ez * qy);
    const float ny = ew * qy + qw * ey + (ez * qx - ex * qz);
    const float nz = ew * qz + qw * ez + (ex * qy - ey * qx);
    const float nrm = sqrtf(nw * nw + nx * nx + ny * ny + nz * nz);
    const float inv = ((nw < 0.f) ? -1.f : 1.f) / nrm;
    newv[cnt][0] = tix + e * phi[0];
    newv[cnt][1] = tiy + e * phi[1];
    newv[cnt][2] = tiz + e * phi[2];
    newv[cnt][3] = nw * inv;
    newv[cnt][4] = nx * inv;
    newv[cnt][5] = ny * inv;
    newv[cnt][6] = nz * inv;
  }
  // poses are read from LDS only, so writing them back to global memory now
  // cannot disturb the other particles' directions
  cnt = 0;
  for (int ii = tid; ii < K; ii += 256, ++cnt)
    for (int a = 0; a < 7; ++a) d.theta[a * Kt + base + ii] = newv[cnt][a];
}

void launch_svgd(const Dev& d, float gamma, float tau, float inv_log_k, hipStream_t s) {
  hipLaunchKernelGGL(k_svgd, dim3(d.G), dim3(256), 0, s, d, gamma, tau, inv_log_k);
}

}  // namespace asicp
