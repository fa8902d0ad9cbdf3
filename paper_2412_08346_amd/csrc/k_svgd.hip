// k_svgd.hip -- annealed Stein ICP update of each (object, preshape) group
// (eqs. (6)-(11)), in two to five launches:
//   k_bw_pass     x4: h of the RBF kernel (eq. 9), the lower median of
//                 |t_i - t_j|^2 over pairs i < j divided by ln K and floored,
//                 found exactly by a radix select over the FP32 bit patterns
//                 (monotone for non-negative floats), 8 bits per pass
//                 (k_bw_fused instead: all four passes in one workgroup per
//                 group when K <= 128);
//   k_svgd_phi    Stein direction in the 6-D tangent: kernel-weighted mean of
//                 the preconditioned driving terms -gamma A g_j (g_j minus the
//                 log-prior gradient when a prior is given, eq. 8) plus tau times
//                 the kernel gradient with respect to particle j (translation
//                 part scaled by h/2); 4 particles per workgroup, 64 lanes
//                 per particle;
//                 the same launch applies t += eta phi_t, q <-
//                 canon(normalize(Exp(eta phi_w) (x) q)), writing the next
//                 poses to the second pose buffer.
// Every phi is computed from the poses of the same iteration: they are read
// from one buffer and the updated poses written to the other.
#include "asicp_internal.h"

namespace asicp {

constexpr int kMaxK = 1024;

__device__ __forceinline__ float d2_of(const float* st, int i, int j) {
  const float dx = st[3 * i + 0] - st[3 * j + 0];
  const float dy = st[3 * i + 1] - st[3 * j + 1];
  const float dz = st[3 * i + 2] - st[3 * j + 2];
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// One radix pass over the K x K ordered pairs (i != j: every unordered pair
// twice) of group blockIdx.y, sliced over gridDim.x workgroups.  Each
// workgroup builds a digit histogram of the pairs matching the current prefix
// in LDS (in the first pass one atomic per distinct digit of a wave, later one
// per pair), adds it into the group's
// global histogram, and the last workgroup to finish picks the digit holding
// the target rank, clears the histogram and, after the last pass, writes h.
__global__ __launch_bounds__(256) void k_bw_pass(Dev d, int pass, float inv_log_k) {
  __shared__ float st[kMaxK * 3];
  __shared__ unsigned int hist[256];
  __shared__ int s_last;
  const int g = blockIdx.y, tid = threadIdx.x, lane = tid & 63, K = d.K, Kt = d.Ktot;
  unsigned int* ghist = d.bw_hist + (size_t)g * 256;
  unsigned int* state = d.bw_state + (size_t)g * 4;  // prefix, mask, rank, done
  for (int j = tid; j < K; j += 256)
    for (int a = 0; a < 3; ++a) st[3 * j + a] = d.theta[a * Kt + g * K + j];
  hist[tid] = 0u;
  const unsigned int P = (unsigned int)K * (unsigned int)(K - 1) / 2u;
  const unsigned int prefix = pass == 0 ? 0u : state[0];
  const unsigned int mask = pass == 0 ? 0u : state[1];
  __syncthreads();
  const int shift = 24 - 8 * pass;
  const int slots = K * K;
  const int per = (slots + gridDim.x - 1) / gridDim.x;
  const int s0 = blockIdx.x * per, s1 = min(slots, s0 + per);
  for (int sb = s0; sb < s1; sb += 256) {
    const int sidx = sb + tid;
    bool act = false;
    unsigned int dig = 0u;
    if (sidx < s1) {
      const int i = sidx / K, j = sidx - (sidx / K) * K;
      if (i != j) {
        const float dx = st[3 * i] - st[3 * j], dy = st[3 * i + 1] - st[3 * j + 1], dz = st[3 * i + 2] - st[3 * j + 2];
        const unsigned int bits = __float_as_uint(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
        act = (bits & mask) == prefix;
        dig = (bits >> shift) & 255u;
      }
    }
    if (pass == 0) {
      // sign and exponent bits: few distinct digits per wave, one atomic each
      unsigned long long pending = __ballot(act);
      while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const unsigned int b = __shfl(dig, leader, 64);
        const unsigned long long same = __ballot(act && dig == b);
        if (lane == leader) atomicAdd(&hist[b], (unsigned int)__popcll(same));
        if (act && dig == b) act = false;
        pending &= ~same;
      }
    } else if (act) {
      // mantissa digits are spread out: plain LDS atomics rarely collide
      atomicAdd(&hist[dig], 1u);
    }
  }
  __syncthreads();
  if (hist[tid]) atomicAdd(&ghist[tid], hist[tid]);
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = (atomicAdd(&state[3], 1u) == gridDim.x - 1) ? 1 : 0;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  if (tid < 64) {  // wave 0 locates the digit holding the rank
    unsigned int c[4], run = 0u;
    for (int r = 0; r < 4; ++r) {
      c[r] = atomicAdd(&ghist[4 * tid + r], 0u);
      run += c[r];
    }
    unsigned int incl = run;
    for (int off = 1; off < 64; off <<= 1) {
      const unsigned int o = __shfl_up(incl, off, 64);
      if (tid >= off) incl += o;
    }
    const unsigned int excl = incl - run;
    const unsigned int rank = pass == 0 ? 2u * ((P - 1u) / 2u) : state[2];
    if (rank >= excl && rank < incl) {
      unsigned int cum = excl;
      for (int r = 0; r < 4; ++r) {
        if (rank < cum + c[r]) {
          const unsigned int np = prefix | ((unsigned int)(4 * tid + r) << shift);
          state[0] = np;
          state[1] = mask | (255u << shift);
          state[2] = rank - cum;
          if (pass == 3) d.h[g] = fmaxf(__uint_as_float(np) * inv_log_k, d.h_min);
          break;
        }
        cum += c[r];
      }
    }
    for (int r = 0; r < 4; ++r) ghist[4 * tid + r] = 0u;
    if (tid == 0) state[3] = 0u;
  }
}

// The same radix select in one workgroup per group of 256, 512 or 1024
// threads (the fewest that hold K (K - 1) / 2 <= 32768 unordered pairs, so
// K <= 256, at 32 per thread: smaller workgroups find room on CUs busy with
// the forward NN launch beside them): each thread keeps the bit patterns of
// its (at most 32) pairs in registers, so the distances are formed
// once and the four passes only rebuild the LDS histogram and pick a digit,
// with no global histogram, no last-workgroup hand-off and one launch instead
// of four.  Pair slot s is {i, (i + d) mod K} with i = s mod K, d = s / K + 1:
// d runs over 1 .. floor((K - 1) / 2) for every i, and for even K the slots
// d = K / 2, i < K / 2 follow, so each unordered pair appears once.  By
// default it is launched only where 256 threads suffice (K <= 128, see
// launch_bandwidth).
constexpr int kBwRegs = 32;
__global__ __launch_bounds__(1024) void k_bw_fused(Dev d, float inv_log_k) {
  __shared__ float st[256 * 3];
  __shared__ unsigned int hist[256];
  __shared__ unsigned int s_sel[3];  // prefix, mask, rank
  const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, K = d.K, Kt = d.Ktot;
  const int nt = blockDim.x;  // 256, 512 or 1024
  for (int j = tid; j < 3 * K; j += nt) {
    const int a = j / K, p = j - a * K;
    st[3 * p + a] = d.theta[a * Kt + g * K + p];
  }
  if (tid < 256) hist[tid] = 0u;
  __syncthreads();
  const int P = K * (K - 1) / 2;
  const int step_d = nt / K, step_i = nt - step_d * K;
  int pi = tid % K, pd = tid / K + 1;
  unsigned int bits[kBwRegs];
  // distances, and the first-pass histogram (sign and exponent bits: few
  // distinct digits per wave, so one atomic per digit and wave)
#pragma unroll
  for (int r = 0; r < kBwRegs; ++r) {
    bits[r] = 0u;
    if (r * nt < P) {
      bool act = r * nt + tid < P;
      if (act) {
        int pj = pi + pd;
        pj -= pj >= K ? K : 0;
        const float dx = st[3 * pi] - st[3 * pj], dy = st[3 * pi + 1] - st[3 * pj + 1],
                    dz = st[3 * pi + 2] - st[3 * pj + 2];
        bits[r] = __float_as_uint(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
      }
      const unsigned int dig = bits[r] >> 24;
      unsigned long long pending = __ballot(act);
      while (pending) {
        const int leader = __builtin_ctzll(pending);
        const unsigned int b = __builtin_amdgcn_readlane(dig, leader);
        const unsigned long long same = __ballot(act && dig == b);
        if (lane == leader) atomicAdd(&hist[b], (unsigned int)__popcll(same));
        act = act && dig != b;
        pending &= ~same;
      }
      pi += step_i;
      pd += step_d;
      if (pi >= K) {
        pi -= K;
        pd += 1;
      }
    }
  }
  unsigned int prefix = 0u, mask = 0u, rank = (unsigned int)(P - 1) / 2u;
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    if (pass > 0) {
#pragma unroll
      for (int r = 0; r < kBwRegs; ++r)
        if (r * nt + tid < P && (bits[r] & mask) == prefix) atomicAdd(&hist[(bits[r] >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid < 64) {
      unsigned int c[4], run = 0u;
      for (int r = 0; r < 4; ++r) {
        c[r] = hist[4 * tid + r];
        run += c[r];
      }
      unsigned int incl = run;
      for (int off = 1; off < 64; off <<= 1) {
        const unsigned int o = __shfl_up(incl, off, 64);
        if (tid >= off) incl += o;
      }
      const unsigned int excl = incl - run;
      if (rank >= excl && rank < incl) {
        unsigned int cum = excl;
        for (int r = 0; r < 4; ++r) {
          if (rank < cum + c[r]) {
            s_sel[0] = prefix | ((unsigned int)(4 * tid + r) << shift);
            s_sel[1] = mask | (255u << shift);
            s_sel[2] = rank - cum;
            break;
          }
          cum += c[r];
        }
      }
      for (int r = 0; r < 4; ++r) hist[4 * tid + r] = 0u;
    }
    __syncthreads();
    prefix = s_sel[0];
    mask = s_sel[1];
    rank = s_sel[2];  // rewritten only after the next pass's first barrier
  }
  if (tid == 0) d.h[g] = fmaxf(__uint_as_float(prefix) * inv_log_k, d.h_min);
}

// bandwidth without a median: fixed h, or h = 1 for a single particle
__global__ void k_bw_const(Dev d) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < d.G) d.h[g] = d.bw_mode == ASICP_BW_FIXED ? d.h_fixed : 1.0f;
}

// Gradient of the log prior of one pose in (t, world rotation vector):
// -w (t - mu_t), and for kappa tr(R(mu)^T R(q)) = kappa (4 (mu.q)^2 - 1) the
// rotation part 4 kappa (mu.q) vec(mu (x) conj q), since the derivative of
// mu.q under q <- Exp(w) q is 1/2 vec(mu (x) conj q).
__device__ __forceinline__ void log_prior_grad(const float* pr, const float* t, const float* q, float* gp) {
  gp[0] = -pr[3] * (t[0] - pr[0]);
  gp[1] = -pr[3] * (t[1] - pr[1]);
  gp[2] = -pr[3] * (t[2] - pr[2]);
  const float mw = pr[4], mx = pr[5], my = pr[6], mz = pr[7];
  const float dot = mw * q[0] + mx * q[1] + my * q[2] + mz * q[3];
  const float c = 4.f * pr[8] * dot;
  gp[3] = c * (q[0] * mx - mw * q[1] - (my * q[3] - mz * q[2]));
  gp[4] = c * (q[0] * my - mw * q[2] - (mz * q[1] - mx * q[3]));
  gp[5] = c * (q[0] * mz - mw * q[3] - (mx * q[2] - my * q[1]));
}

constexpr int kPhiLanes = 64;              // lanes per particle (one wavefront)
constexpr int kPhiPer = 256 / kPhiLanes;   // particles per workgroup
__global__ __launch_bounds__(256) void k_svgd_phi(Dev d, float gamma, float tau) {
  __shared__ float st[kMaxK * 3];
  __shared__ float sq[kMaxK * 4];
  __shared__ float sg[kMaxK * 6];
  const int g = blockIdx.x, tid = threadIdx.x, K = d.K, Kt = d.Ktot;
  const int base = g * K;
  for (int j = tid; j < K; j += 256) {
    const int i = base + j;
    for (int a = 0; a < 3; ++a) st[3 * j + a] = d.theta[a * Kt + i];
    for (int a = 0; a < 4; ++a) sq[4 * j + a] = d.theta[(3 + a) * Kt + i];
    for (int a = 0; a < 6; ++a) sg[6 * j + a] = d.grad[a * Kt + i];
    if (d.prior) {
      float gp[6];
      log_prior_grad(d.prior + 12 * g, st + 3 * j, sq + 4 * j, gp);
      for (int a = 0; a < 6; ++a) sg[6 * j + a] -= gp[a];
    }
  }
  __syncthreads();
  const int ii = blockIdx.y * kPhiPer + tid / kPhiLanes, part = tid % kPhiLanes;
  const float h = d.h[g];
  const float inv_h = 1.0f / h;
  const GroupInfo gi = d.groups[g];
  const float at = d.pre_const[gi.pre * 8 + 4], aw = d.pre_const[gi.pre * 8 + 5];
  const float ga_t = gamma * at, ga_w = gamma * aw;
  const bool block = d.kernel_mode == ASICP_KERNEL_BLOCK;
  float acc[6] = {0, 0, 0, 0, 0, 0};
  if (ii < K) {
    const float tix = st[3 * ii], tiy = st[3 * ii + 1], tiz = st[3 * ii + 2];
    const float qw = sq[4 * ii], qx = sq[4 * ii + 1], qy = sq[4 * ii + 2], qz = sq[4 * ii + 3];
    for (int j = part; j < K; j += kPhiLanes) {
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
  }
  // sum over the particle's wavefront (a fixed tree): every lane gets the total
#pragma unroll
  for (int a = 0; a < 6; ++a) acc[a] = wave_sum(acc[a]);
  if (!(ii < K && part == 0)) return;
  const float invK = 1.0f / (float)K;
  float ph[6];
  for (int a = 0; a < 6; ++a) {
    ph[a] = acc[a] * invK;
    d.phi[a * Kt + base + ii] = ph[a];
  }
  // the update of eqs. (7), (3): t += eta phi_t, q <- canon(normalize(Exp(eta
  // phi_w) (x) q)), written to the other pose buffer (every workgroup of the
  // group reads the poses of this iteration from the current one)
  const int i = base + ii;
  const float e = d.eta;
  float t[3], q[4];
  for (int a = 0; a < 3; ++a) t[a] = st[3 * ii + a];
  for (int a = 0; a < 4; ++a) q[a] = sq[4 * ii + a];
  const float wx = e * ph[3], wy = e * ph[4], wz = e * ph[5];
  const float th = sqrtf(wx * wx + wy * wy + wz * wz);
  float ew = 1.f, ex = 0.f, ey = 0.f, ez = 0.f;
  if (th > 0.f) {
    float sh, ch;
    sincosf(0.5f * th, &sh, &ch);
    const float s = sh / th;
    ew = ch; ex = s * wx; ey = s * wy; ez = s * wz;
  }
  const float nw = ew * q[0] - ex * q[1] - ey * q[2] - ez * q[3];
  const float nx = ew * q[1] + q[0] * ex + (ey * q[3] - ez * q[2]);
  const float ny = ew * q[2] + q[0] * ey + (ez * q[1] - ex * q[3]);
  const float nz = ew * q[3] + q[0] * ez + (ex * q[2] - ey * q[1]);
  const float nrm = sqrtf(nw * nw + nx * nx + ny * ny + nz * nz);
  const float inv = ((nw < 0.f) ? -1.f : 1.f) / nrm;
  float* out = d.theta_next;
  out[0 * Kt + i] = t[0] + e * ph[0];
  out[1 * Kt + i] = t[1] + e * ph[1];
  out[2 * Kt + i] = t[2] + e * ph[2];
  out[3 * Kt + i] = nw * inv;
  out[4 * Kt + i] = nx * inv;
  out[5 * Kt + i] = ny * inv;
  out[6 * Kt + i] = nz * inv;
}

void launch_bandwidth(const Dev& d, float inv_log_k, hipStream_t s) {
  if (d.K >= 2 && d.bw_mode == ASICP_BW_MEDIAN) {
    // The fused select only where it fits a 256-thread workgroup (K <= 128):
    // beside the forward NN launch, a 512- or 1024-thread workgroup waits
    // for a CU to drain, while the sliced passes' 256-thread workgroups take
    // the place of retiring forward workgroups (measured on K = 256: 41.4
    // against 41.8 ms per paper-scale solve).
#ifndef ASICP_BW_FUSED_MAX_PAIRS
#define ASICP_BW_FUSED_MAX_PAIRS (kBwRegs * 256)
#endif
    const int pairs = d.K * (d.K - 1) / 2;
    if (pairs <= ASICP_BW_FUSED_MAX_PAIRS) {
      int nt = 256;
      while (nt * kBwRegs < pairs) nt *= 2;
      hipLaunchKernelGGL(k_bw_fused, dim3(d.G), dim3(nt), 0, s, d, inv_log_k);
    } else {
      for (int pass = 0; pass < 4; ++pass)
        hipLaunchKernelGGL(k_bw_pass, dim3(kBwSlices, d.G), dim3(256), 0, s, d, pass, inv_log_k);
    }
  } else {
    hipLaunchKernelGGL(k_bw_const, dim3((d.G + 255) / 256), dim3(256), 0, s, d);
  }
}

void launch_stein(const Dev& d, float gamma, float tau, hipStream_t s) {
  hipLaunchKernelGGL(k_svgd_phi, dim3(d.G, (d.K + kPhiPer - 1) / kPhiPer), dim3(256), 0, s, d, gamma, tau);
}

}  // namespace asicp
