// k_proposal.hip -- learned grasp proposal: a max-pooled point-cloud encoder
// (PointNet style) that maps an object cloud to S seed poses per preshape for
// the AS-ICP iteration.  The paper points to learned priors and data-driven
// seeding as the way to need fewer initialisations (Sec. V, the
// ablation; Sec. VII); the network, its loss and its training are this library's.
//
//   x_m  = (r_m - mean r) / 0.1
//   h1_m = relu(W1 x_m + b1)          3 -> 64      (VALU, FP32)
//   h2_m = relu(W2 h1_m + b2)        64 -> 128     (BF16 MFMA, FP32 accumulate)
//   h3_m = relu(W3 h2_m + b3)       128 -> 256     (BF16 MFMA, FP32 accumulate)
//   g    = max_m h3_m                (lowest m on ties)
//   u = relu(W4 g + b4), v = relu(W5 u + b5), o = W6 v + b6   (FP32)
//   seed (p, s): t = mean r + 0.1 o[0:3], q = o[3:7] / |o[3:7]|
//
// Loss per (object, preshape) against T target poses (t_g, q_g):
//   d(a, g) = |t_a - t_g|^2 / 0.01 + (1 - (q_a . q_g)^2),
//   L = (1/T) sum_g min_a d + (1/S) sum_a min_g d, averaged over preshapes and
//   objects.  The max-pool routes each channel's gradient to one point, so
//   the encoder's backward touches at most 256 points per object: their
//   products run on BF16 MFMA with FP32 accumulation (k_pn_point_bwd).
// Every sum runs in a fixed order: no float atomics.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "asicp_internal.h"

namespace asicp {

namespace pn {

constexpr int H1 = 64, H2 = 128, H3 = 256, HH = 256;
constexpr float kUnit = 0.1f;
constexpr int kPts = 64;  // points per forward workgroup

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct Params {  // offsets (floats) into the flat parameter array
  int W1, b1, W2, b2, W3, b3, W4, b4, W5, b5, W6, b6, total, O;
};

__host__ __device__ inline Params layout(int n_pre, int n_seed) {
  Params p;
  int o = 0;
  p.O = n_pre * n_seed * 7;
  p.W1 = o; o += H1 * 3;
  p.b1 = o; o += H1;
  p.W2 = o; o += H2 * H1;
  p.b2 = o; o += H2;
  p.W3 = o; o += H3 * H2;
  p.b3 = o; o += H3;
  p.W4 = o; o += HH * H3;
  p.b4 = o; o += HH;
  p.W5 = o; o += HH * HH;
  p.b5 = o; o += HH;
  p.W6 = o; o += p.O * HH;
  p.b6 = o; o += p.O;
  p.total = o;
  return p;
}

// FP32 -> BF16, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

struct Net {
  const float* prm;           // flat FP32 parameters
  unsigned short* w2h;        // BF16 copy of W2 [128][64]
  unsigned short* w3h;        // BF16 copy of W3 [256][128]
  const int32_t* off;         // [n_obj + 1] point offsets
  const float *x, *y, *z;     // clouds, SoA
  float* com;                 // [n_obj][4] centroid
  unsigned long long* pool;   // [n_obj][256] (value bits << 32) | ~index, max
  float* head;                // [n_obj][4][256] g, u, v (post-activation), spare
  float* out;                 // [n_obj][O] raw outputs
  float* dout;                // [n_obj][O] dL/do
  float* dhead;               // [n_obj][3][256] dzv, dzu, dg
  float* part;                // [n_obj][n_enc] per-object encoder gradient
  int n_obj, n_pre, n_seed, n_tgt;
  Params P;
};

constexpr int kEnc = H1 * 3 + H1 + H2 * H1 + H2 + H3 * H2 + H3;  // encoder parameters

// ---------------------------------------------------------------------------
// set-up: BF16 weights, pool reset, centroids (FP64 in a fixed order)
__global__ __launch_bounds__(256) void k_pn_prep(Net n) {
  const int tid = threadIdx.x, bid = blockIdx.x;
  if (bid == 0) {
    for (int i = tid; i < H2 * H1; i += 256) n.w2h[i] = to_bf16(n.prm[n.P.W2 + i]);
    for (int i = tid; i < H3 * H2; i += 256) n.w3h[i] = to_bf16(n.prm[n.P.W3 + i]);
    return;
  }
  const int o = bid - 1;
  if (o >= n.n_obj) return;
  __shared__ double s[3][256];
  const int a = n.off[o], b = n.off[o + 1];
  double sx = 0, sy = 0, sz = 0;
  for (int i = a + tid; i < b; i += 256) { sx += n.x[i]; sy += n.y[i]; sz += n.z[i]; }
  s[0][tid] = sx; s[1][tid] = sy; s[2][tid] = sz;
  n.pool[(size_t)o * H3 + tid] = 0ull;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st)
      for (int c = 0; c < 3; ++c) s[c][tid] += s[c][tid + st];
    __syncthreads();
  }
  if (tid < 3) n.com[o * 4 + tid] = (float)(s[tid][0] / (double)(b - a));
}

// ---------------------------------------------------------------------------
// forward of the point MLP for 64 points of one object and the max-pool
__global__ __launch_bounds__(256) void k_pn_point_fwd(Net n, int chunks_per_obj) {
  __shared__ unsigned short a1[kPts][H1 + 4];   // BF16 h1, row = point (padded rows)
  __shared__ unsigned short a2[kPts][H2 + 4];   // BF16 h2
  __shared__ float xs[kPts][3];
  const int o = blockIdx.x / chunks_per_obj, ch = blockIdx.x - o * chunks_per_obj;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int a = n.off[o], b = n.off[o + 1];
  const int p0 = a + ch * kPts;
  if (p0 >= b) return;  // uniform over the workgroup
  const int np = min(kPts, b - p0);
  if (tid < kPts) {
    // rows past the cloud repeat its first point of this chunk: they take part
    // in the products but never in the max (masked below)
    const int i = p0 + (tid < np ? tid : 0);
    xs[tid][0] = (n.x[i] - n.com[o * 4 + 0]) / kUnit;
    xs[tid][1] = (n.y[i] - n.com[o * 4 + 1]) / kUnit;
    xs[tid][2] = (n.z[i] - n.com[o * 4 + 2]) / kUnit;
  }
  __syncthreads();
  // layer 1: 64 points x 64 channels, 16 per thread
  for (int e = tid; e < kPts * H1; e += 256) {
    const int m = e / H1, c = e - m * H1;
    const float* W1 = n.prm + n.P.W1 + c * 3;
    float zz = n.prm[n.P.b1 + c];
    zz = __builtin_fmaf(W1[0], xs[m][0], zz);
    zz = __builtin_fmaf(W1[1], xs[m][1], zz);
    zz = __builtin_fmaf(W1[2], xs[m][2], zz);
    a1[m][c] = to_bf16(fmaxf(zz, 0.f));
  }
  __syncthreads();
  const int row = lane & 15, kq = lane >> 4;  // A: row m, k block kq; B: column n, k block kq
  // layer 2: [64 x 64] . [64 x 128]; wave w takes output column tiles 2w, 2w+1
  for (int nt = 2 * w; nt < 2 * w + 2; ++nt) {
    for (int mt = 0; mt < kPts / 16; ++mt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < H1; k0 += 16) {
        s4 av, bv;
        const unsigned short* ap = &a1[mt * 16 + row][k0 + 4 * kq];
        const unsigned short* bp = n.w2h + (size_t)(nt * 16 + row) * H1 + k0 + 4 * kq;
#pragma unroll
        for (int j = 0; j < 4; ++j) { av[j] = (short)ap[j]; bv[j] = (short)bp[j]; }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
      // D[row = 4 kq + v][col = lane % 16]: point mt*16 + 4kq + v, channel nt*16 + lane%16
      const int c = nt * 16 + row;
      const float bias = n.prm[n.P.b2 + c];
#pragma unroll
      for (int v = 0; v < 4; ++v) a2[mt * 16 + 4 * kq + v][c] = to_bf16(fmaxf(acc[v] + bias, 0.f));
    }
  }
  __syncthreads();
  // layer 3: [64 x 128] . [128 x 256] and the max over the chunk's points;
  // wave w takes output column tiles 4w .. 4w+3
  for (int nt = 4 * w; nt < 4 * w + 4; ++nt) {
    const int c = nt * 16 + row;
    const float bias = n.prm[n.P.b3 + c];
    unsigned long long best = 0ull;
    for (int mt = 0; mt < kPts / 16; ++mt) {
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int k0 = 0; k0 < H2; k0 += 16) {
        s4 av, bv;
        const unsigned short* ap = &a2[mt * 16 + row][k0 + 4 * kq];
        const unsigned short* bp = n.w3h + (size_t)(nt * 16 + row) * H2 + k0 + 4 * kq;
#pragma unroll
        for (int j = 0; j < 4; ++j) { av[j] = (short)ap[j]; bv[j] = (short)bp[j]; }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = mt * 16 + 4 * kq + v;
        if (m < np) {
          const float h = fmaxf(acc[v] + bias, 0.f);
          // larger value wins; on equal values the lower point index
          const unsigned long long key =
              ((unsigned long long)__float_as_uint(h) << 32) | (0xFFFFFFFFu - (unsigned)(p0 + m - a));
          best = key > best ? key : best;
        }
      }
    }
    // combine the four lane groups (rows) of each column
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const unsigned long long other = __shfl_xor(best, off, 64);
      best = other > best ? other : best;
    }
    if (lane < 16 && best) atomicMax(n.pool + (size_t)o * H3 + c, best);
  }
}

// ---------------------------------------------------------------------------
// head: g -> u -> v -> o, and the seed poses (SoA, solver order)
__global__ __launch_bounds__(256) void k_pn_head_fwd(Net n, float* seeds, int Ktot, float retract) {
  __shared__ float g[H3], u[HH], v[HH];
  const int o = blockIdx.x, tid = threadIdx.x;
  const unsigned long long key = n.pool[(size_t)o * H3 + tid];
  g[tid] = __uint_as_float((unsigned)(key >> 32));
  __syncthreads();
  {
    const float* W = n.prm + n.P.W4 + (size_t)tid * H3;
    float acc = n.prm[n.P.b4 + tid];
    for (int k = 0; k < H3; ++k) acc = __builtin_fmaf(W[k], g[k], acc);
    u[tid] = fmaxf(acc, 0.f);
  }
  __syncthreads();
  {
    const float* W = n.prm + n.P.W5 + (size_t)tid * HH;
    float acc = n.prm[n.P.b5 + tid];
    for (int k = 0; k < HH; ++k) acc = __builtin_fmaf(W[k], u[k], acc);
    v[tid] = fmaxf(acc, 0.f);
  }
  __syncthreads();
  float* hd = n.head + (size_t)o * 4 * 256;
  hd[tid] = g[tid];
  hd[256 + tid] = u[tid];
  hd[512 + tid] = v[tid];
  const int O = n.P.O;
  for (int r = tid; r < O; r += 256) {
    const float* W = n.prm + n.P.W6 + (size_t)r * HH;
    float acc = n.prm[n.P.b6 + r];
    for (int k = 0; k < HH; ++k) acc = __builtin_fmaf(W[k], v[k], acc);
    n.out[(size_t)o * O + r] = acc;
  }
  if (!seeds) return;
  __syncthreads();
  const int ns = n.n_pre * n.n_seed;
  for (int j = tid; j < ns; j += 256) {
    const float* r = n.out + (size_t)o * O + (size_t)j * 7;
    const int i = o * ns + j;  // particle index: (object, preshape, seed)
    for (int a = 0; a < 3; ++a) seeds[(size_t)a * Ktot + i] = n.com[o * 4 + a] + kUnit * r[a];
    float qw = r[3], qx = r[4], qy = r[5], qz = r[6];
    const float nrm = sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    const float s = (qw < 0.f ? -1.f : 1.f) / (nrm > 0.f ? nrm : 1.f);
    if (nrm > 0.f) {
      qw *= s; qx *= s; qy *= s; qz *= s;
    } else {
      qw = 1.f; qx = qy = qz = 0.f;
    }
    seeds[(size_t)3 * Ktot + i] = qw;
    seeds[(size_t)4 * Ktot + i] = qx;
    seeds[(size_t)5 * Ktot + i] = qy;
    seeds[(size_t)6 * Ktot + i] = qz;
    // back the gripper off along its approach axis (third column of R(q))
    const float ax = 2.f * (qx * qz + qw * qy), ay = 2.f * (qy * qz - qw * qx), az = 1.f - 2.f * (qx * qx + qy * qy);
    seeds[(size_t)0 * Ktot + i] -= retract * ax;
    seeds[(size_t)1 * Ktot + i] -= retract * ay;
    seeds[(size_t)2 * Ktot + i] -= retract * az;
  }
}

// ---------------------------------------------------------------------------
// set loss and dL/do: one wave per (object, preshape).  The lanes split the
// targets (nearest seed of each, lowest index on ties), then the seeds
// (nearest target of each); each seed's gradient is accumulated by its own
// lane in the order target 0 .. T-1, then its own nearest target, and the
// loss is summed by lane 0 in the order targets, then seeds.
constexpr int kLossMaxS = 1024 / 7;  // seeds per preshape (n_pre * n_seed * 7 <= 1024)
constexpr int kLossMaxT = 4096;      // targets per preshape
__global__ __launch_bounds__(64) void k_pn_loss(Net n, const float* tgt, float* lpart) {
  __shared__ float sd[kLossMaxS][8];  // seed: t (3, metres), q / |q| (4), 1 / |q|
  __shared__ int bs_of[kLossMaxT];    // nearest seed of each target
  __shared__ float bd_t[kLossMaxT], bd_s[kLossMaxS];
  const int j = blockIdx.x, lane = threadIdx.x;
  const int o = j / n.n_pre, p = j - o * n.n_pre;
  const int S = n.n_seed, T = n.n_tgt, O = n.P.O;
  const float* a = n.out + (size_t)o * O + (size_t)p * S * 7;
  float* da = n.dout + (size_t)o * O + (size_t)p * S * 7;
  const float* tg = tgt + ((size_t)o * n.n_pre + p) * T * 7;
  const float cx = n.com[o * 4], cy = n.com[o * 4 + 1], cz = n.com[o * 4 + 2];
  for (int s = lane; s < S; s += 64) {
    const float* r = a + s * 7;
    sd[s][0] = cx + kUnit * r[0];
    sd[s][1] = cy + kUnit * r[1];
    sd[s][2] = cz + kUnit * r[2];
    const float nq = sqrtf(r[3] * r[3] + r[4] * r[4] + r[5] * r[5] + r[6] * r[6]);
    for (int e = 0; e < 4; ++e) sd[s][3 + e] = r[3 + e] / nq;
    sd[s][7] = 1.f / nq;
  }
  __syncthreads();
  // d(a, g) = |t_a - t_g|^2 / UNIT^2 + 1 - (q_a . q_g)^2 and q_a . q_g
  auto dist = [&](int s, const float* t, float* c_out) {
    const float dx = sd[s][0] - t[0], dy = sd[s][1] - t[1], dz = sd[s][2] - t[2];
    const float c = sd[s][3] * t[3] + sd[s][4] * t[4] + sd[s][5] * t[5] + sd[s][6] * t[6];
    *c_out = c;
    return (dx * dx + dy * dy + dz * dz) / (kUnit * kUnit) + (1.f - c * c);
  };
  float c;
  for (int g = lane; g < T; g += 64) {
    const float* t = tg + g * 7;
    int bs = 0;
    float bd = dist(0, t, &c);
    for (int s = 1; s < S; ++s) {
      const float dd = dist(s, t, &c);
      if (dd < bd) { bd = dd; bs = s; }
    }
    bs_of[g] = bs;
    bd_t[g] = bd;
  }
  __syncthreads();
  const float w_t = 1.f / (float)T / (float)n.n_pre, w_s = 1.f / (float)S / (float)n.n_pre;
  for (int s = lane; s < S; s += 64) {
    float d[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // adds wgt * dd(s, g) / d(raw seed s)
    auto grad = [&](const float* t, float wgt) {
      const float dx = sd[s][0] - t[0], dy = sd[s][1] - t[1], dz = sd[s][2] - t[2];
      const float f = wgt * 2.f / kUnit;  // d/d raw t = 2 dt / UNIT^2 * UNIT
      d[0] += f * dx; d[1] += f * dy; d[2] += f * dz;
      const float cc = sd[s][3] * t[3] + sd[s][4] * t[4] + sd[s][5] * t[5] + sd[s][6] * t[6];
      const float k = -2.f * wgt * cc * sd[s][7];
      for (int e = 0; e < 4; ++e) d[3 + e] += k * (t[3 + e] - cc * sd[s][3 + e]);
    };
    for (int g = 0; g < T; ++g)
      if (bs_of[g] == s) grad(tg + g * 7, w_t);
    int bg = 0;
    float bd = dist(s, tg, &c);
    for (int g = 1; g < T; ++g) {
      const float dd = dist(s, tg + g * 7, &c);
      if (dd < bd) { bd = dd; bg = g; }
    }
    grad(tg + bg * 7, w_s);
    bd_s[s] = bd;
    for (int e = 0; e < 7; ++e) da[s * 7 + e] = d[e];
  }
  __syncthreads();
  if (lane == 0) {
    float L = 0.f;
    for (int g = 0; g < T; ++g) L += bd_t[g] / (float)T;
    for (int s = 0; s < S; ++s) L += bd_s[s] / (float)S;
    lpart[j] = L / (float)n.n_pre;
  }
}

// per object: loss over preshapes (fixed order)
__global__ void k_pn_loss_sum(Net n, const float* lpart, float* loss) {
  const int o = blockIdx.x * 64 + threadIdx.x;
  if (o >= n.n_obj) return;
  float L = 0.f;
  for (int p = 0; p < n.n_pre; ++p) L += lpart[o * n.n_pre + p];
  loss[o] = L;
}

// ---------------------------------------------------------------------------
// head backward per object: dzv, dzu, dg
__global__ __launch_bounds__(256) void k_pn_head_bwd(Net n) {
  __shared__ float dov[1024];
  __shared__ float dzv[HH], dzu[HH];
  const int o = blockIdx.x, tid = threadIdx.x, O = n.P.O;
  const float* hd = n.head + (size_t)o * 4 * 256;
  float* dh = n.dhead + (size_t)o * 3 * 256;
  for (int r = tid; r < O; r += 256) dov[r] = n.dout[(size_t)o * O + r];
  __syncthreads();
  {  // dv = W6^T do, through the relu of v
    float acc = 0.f;
    for (int r = 0; r < O; ++r) acc = __builtin_fmaf(n.prm[n.P.W6 + (size_t)r * HH + tid], dov[r], acc);
    dzv[tid] = hd[512 + tid] > 0.f ? acc : 0.f;
  }
  __syncthreads();
  {
    float acc = 0.f;
    for (int r = 0; r < HH; ++r) acc = __builtin_fmaf(n.prm[n.P.W5 + (size_t)r * HH + tid], dzv[r], acc);
    dzu[tid] = hd[256 + tid] > 0.f ? acc : 0.f;
  }
  __syncthreads();
  float acc = 0.f;
  for (int r = 0; r < HH; ++r) acc = __builtin_fmaf(n.prm[n.P.W4 + (size_t)r * H3 + tid], dzu[r], acc);
  dh[tid] = dzv[tid];
  dh[256 + tid] = dzu[tid];
  dh[512 + tid] = acc;  // dL/dg
}

// head weight gradients: sums over objects in a fixed order, one element per
// thread; the result is divided by the number of objects (mean loss)
__global__ __launch_bounds__(256) void k_pn_head_wgrad(Net n, float* grad) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  const int O = n.P.O;
  const long long n4 = (long long)HH * H3, n5 = (long long)HH * HH, n6 = (long long)O * HH;
  const long long tot = n4 + HH + n5 + HH + n6 + O;
  if (e >= tot) return;
  const float inv = 1.f / (float)n.n_obj;
  float acc = 0.f;
  long long r = e;
  if (r < n4) {
    const int i = (int)(r / H3), k = (int)(r - (long long)i * H3);
    for (int o = 0; o < n.n_obj; ++o)
      acc = __builtin_fmaf(n.dhead[(size_t)o * 768 + 256 + i], n.head[(size_t)o * 1024 + k], acc);
    grad[n.P.W4 + r] = acc * inv;
    return;
  }
  r -= n4;
  if (r < HH) {
    for (int o = 0; o < n.n_obj; ++o) acc += n.dhead[(size_t)o * 768 + 256 + r];
    grad[n.P.b4 + r] = acc * inv;
    return;
  }
  r -= HH;
  if (r < n5) {
    const int i = (int)(r / HH), k = (int)(r - (long long)i * HH);
    for (int o = 0; o < n.n_obj; ++o)
      acc = __builtin_fmaf(n.dhead[(size_t)o * 768 + i], n.head[(size_t)o * 1024 + 256 + k], acc);
    grad[n.P.W5 + r] = acc * inv;
    return;
  }
  r -= n5;
  if (r < HH) {
    for (int o = 0; o < n.n_obj; ++o) acc += n.dhead[(size_t)o * 768 + r];
    grad[n.P.b5 + r] = acc * inv;
    return;
  }
  r -= HH;
  if (r < n6) {
    const int i = (int)(r / HH), k = (int)(r - (long long)i * HH);
    for (int o = 0; o < n.n_obj; ++o)
      acc = __builtin_fmaf(n.dout[(size_t)o * O + i], n.head[(size_t)o * 1024 + 512 + k], acc);
    grad[n.P.W6 + r] = acc * inv;
    return;
  }
  r -= n6;
  for (int o = 0; o < n.n_obj; ++o) acc += n.dout[(size_t)o * O + r];
  grad[n.P.b6 + r] = acc * inv;
}

// ---------------------------------------------------------------------------
// encoder backward, one workgroup per object.  Channel c's gradient dg_c goes
// to its argmax point p_c (where h3 = g_c > 0, so the relu passes it); the
// distinct routed points (at most 256) form the rows of the products below,
// processed in tiles of 64 rows:
//   forward recompute   z1 (VALU, the forward's FMA order), h1 = bf16 relu(z1),
//                       z2 = h1 W2^T + b2 (the forward's BF16 MFMA, so the
//                       relu masks are the forward's bit for bit),
//                       h2 = bf16 relu(z2);
//   dW3 row c, db3 c    dg_c h2[p_c] (one point per channel: outer products);
//   dh2                 sum over the row's channels of dg_c W3[c] (gather);
//   dz2                 dh2 where z2 > 0, split into BF16 hi + lo parts
//                       (|dz2 - hi - lo| <= 2^-17 |dz2|);
//   dW2 += dz2^T h1     BF16 MFMA over the rows, hi and lo, FP32 accumulate
//                       (kept in registers across the tiles);
//   dh1 = dz2 W2        BF16 MFMA over the 128 channels, hi and lo;
//   dz1                 dh1 where z1 > 0;  dW1 += dz1^T x, db1, db2 (VALU).
// Every sum runs in a fixed order; the record of the object is written once.
constexpr int kBwdRows = 64;  // routed points per tile
__global__ __launch_bounds__(256) void k_pn_point_bwd(Net n) {
  __shared__ unsigned int keyp[H3];   // (point << 8) | channel, sorted; 0xFFFFFFFF = no gradient
  __shared__ float dgs[H3];
  __shared__ int seg_row[H3];         // sorted position -> row (distinct point)
  __shared__ int row_first[H3 + 1];   // row -> first sorted position of its channels
  __shared__ int row_pt[H3];          // row -> point index in the object
  __shared__ int n_rows;
  __shared__ float xs[kBwdRows][3];
  __shared__ unsigned short a1s[kBwdRows][H1 + 4];  // bf16 h1
  __shared__ unsigned short dzh[kBwdRows][H2 + 2];  // dz2, bf16 hi part
  __shared__ unsigned short dzl[kBwdRows][H2 + 2];  // dz2, bf16 lo part
  // bf16 h2 of the tile, then (once dz2 is formed) dz1 as FP32
  __shared__ __align__(16) unsigned char u2[kBwdRows * (H2 + 4) * 2];
  unsigned short (*a2s)[H2 + 4] = reinterpret_cast<unsigned short (*)[H2 + 4]>(u2);
  float (*dz1s)[H1 + 1] = reinterpret_cast<float (*)[H1 + 1]>(u2);
  static_assert(kBwdRows * (H1 + 1) * 4 <= kBwdRows * (H2 + 4) * 2, "dz1 fits the h2 buffer");

  const int o = blockIdx.x, tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int row = lane & 15, kq = lane >> 4;
  const int a = n.off[o];
  float* part = n.part + (size_t)o * kEnc;
  // encoder record layout: W1, b1, W2, b2, W3, b3 (as in the parameters)
  const int oW1 = 0, ob1 = H1 * 3, oW2 = ob1 + H1, ob2 = oW2 + H2 * H1, oW3 = ob2 + H2, ob3 = oW3 + H3 * H2;
  {
    const unsigned long long key = n.pool[(size_t)o * H3 + tid];
    const float gval = __uint_as_float((unsigned)(key >> 32));
    const float dg = n.dhead[(size_t)o * 768 + 512 + tid];
    const bool live = key != 0ull && gval > 0.f && dg != 0.f;
    const unsigned pt = 0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull);
    keyp[tid] = live ? ((pt << 8) | (unsigned)tid) : 0xFFFFFFFFu;
    dgs[tid] = dg;
    if (!live) {  // channels without gradient: zero rows of dW3 and db3
      for (int i = 0; i < H2; ++i) part[oW3 + tid * H2 + i] = 0.f;
      part[ob3 + tid] = 0.f;
    }
  }
  __syncthreads();
  // bitonic sort of the 256 keys (point major, channel minor)
  for (int size = 2; size <= H3; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int i = tid, j = i ^ stride;
      if (j > i) {
        const bool asc = (i & size) == 0;
        const unsigned ki = keyp[i], kj = keyp[j];
        if ((ki > kj) == asc) { keyp[i] = kj; keyp[j] = ki; }
      }
      __syncthreads();
    }
  }
  // rows: one per distinct point, in point order (a prefix count of the
  // positions that start a new point)
  if (tid == 0) {
    int r = -1;
    unsigned prev = 0xFFFFFFFFu;
    for (int s = 0; s < H3; ++s) {
      const unsigned k = keyp[s];
      if (k == 0xFFFFFFFFu) {
        seg_row[s] = -1;
        continue;
      }
      if ((k >> 8) != prev) {
        ++r;
        row_first[r] = s;
        row_pt[r] = (int)(k >> 8);
        prev = k >> 8;
      }
      seg_row[s] = r;
    }
    int end = 0;
    while (end < H3 && keyp[end] != 0xFFFFFFFFu) ++end;
    row_first[r + 1] = end;
    n_rows = r + 1;
  }
  __syncthreads();
  const int P = n_rows;
  // dW2 accumulators: wave w owns output rows (channels of h2) 32w .. 32w+31
  // as two 16-row tiles, times the four 16-column tiles of h1's channels
  f4 acc2[2][4];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) acc2[mi][ni] = f4{0.f, 0.f, 0.f, 0.f};
  float gW1[3] = {0.f, 0.f, 0.f}, gb1 = 0.f, gb2 = 0.f;  // threads < 64: h1 channel tid; gb2: tid & 127 (half tid >> 7)

  for (int r0 = 0; r0 < P; r0 += kBwdRows) {
    const int nr = min(kBwdRows, P - r0);
    // x and h1 of the tile's rows (rows past the last point are zero)
    if (tid < kBwdRows) {
      for (int c = 0; c < 3; ++c) xs[tid][c] = 0.f;
      if (tid < nr) {
        const int gi = a + row_pt[r0 + tid];
        xs[tid][0] = (n.x[gi] - n.com[o * 4 + 0]) / kUnit;
        xs[tid][1] = (n.y[gi] - n.com[o * 4 + 1]) / kUnit;
        xs[tid][2] = (n.z[gi] - n.com[o * 4 + 2]) / kUnit;
      }
    }
    __syncthreads();
    for (int e = tid; e < kBwdRows * H1; e += 256) {
      const int m = e / H1, c = e - m * H1;
      unsigned short h = 0;
      if (m < nr) {
        const float* W1 = n.prm + n.P.W1 + c * 3;
        float zz = n.prm[n.P.b1 + c];
        zz = __builtin_fmaf(W1[0], xs[m][0], zz);
        zz = __builtin_fmaf(W1[1], xs[m][1], zz);
        zz = __builtin_fmaf(W1[2], xs[m][2], zz);
        h = to_bf16(fmaxf(zz, 0.f));
      }
      a1s[m][c] = h;
    }
    __syncthreads();
    // z2 = h1 W2^T + b2 and h2 = bf16 relu(z2): the forward's products;
    // wave w takes output column tiles 2w, 2w+1
    for (int nt = 2 * w; nt < 2 * w + 2; ++nt) {
      for (int mt = 0; mt < kBwdRows / 16; ++mt) {
        f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int k0 = 0; k0 < H1; k0 += 16) {
          s4 av, bv;
          const unsigned short* ap = &a1s[mt * 16 + row][k0 + 4 * kq];
          const unsigned short* bp = n.w2h + (size_t)(nt * 16 + row) * H1 + k0 + 4 * kq;
#pragma unroll
          for (int j = 0; j < 4; ++j) { av[j] = (short)ap[j]; bv[j] = (short)bp[j]; }
          acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
        }
        const int c = nt * 16 + row;
        const float bias = n.prm[n.P.b2 + c];
#pragma unroll
        for (int v = 0; v < 4; ++v) a2s[mt * 16 + 4 * kq + v][c] = to_bf16(fmaxf(acc[v] + bias, 0.f));
      }
    }
    __syncthreads();
    // dW3 rows and db3 of the tile's channels: two channels per pass
    {
      const int s_begin = row_first[r0], s_end = row_first[r0 + nr];
      for (int s = s_begin + (tid >> 7); s < s_end; s += 2) {
        const int c = (int)(keyp[s] & 255u);
        const int rr = seg_row[s] - r0;
        const int i = tid & 127;
        part[oW3 + c * H2 + i] = dgs[c] * from_bf16(a2s[rr][i]);
        if (i == 0) part[ob3 + c] = dgs[c];
      }
    }
    // dz2 = (sum over the row's channels of dg_c W3[c]) where z2 > 0, as hi +
    // lo BF16; thread tid owns channel tid & 127 of rows (tid >> 7) + 2j
    {
      const int i = tid & 127;
      for (int m = tid >> 7; m < kBwdRows; m += 2) {
        float dz = 0.f;
        if (m < nr && from_bf16(a2s[m][i]) > 0.f) {  // z2 > 0
          float dh = 0.f;
          for (int s = row_first[r0 + m]; s < row_first[r0 + m + 1]; ++s) {
            const int c = (int)(keyp[s] & 255u);
            dh = __builtin_fmaf(from_bf16(n.w3h[(size_t)c * H2 + i]), dgs[c], dh);
          }
          dz = dh;
        }
        gb2 += dz;
        const unsigned short hi = to_bf16(dz);
        dzh[m][i] = hi;
        dzl[m][i] = to_bf16(dz - from_bf16(hi));
      }
    }
    __syncthreads();
    // dW2 += dz2^T h1 over the tile's rows (K = 64 rows in 4 steps, hi and lo)
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const int ch = (2 * w + mi) * 16 + row;  // A row: channel of h2
#pragma unroll
      for (int k0 = 0; k0 < kBwdRows; k0 += 16) {
        s4 ah, al;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ah[j] = (short)dzh[k0 + 4 * kq + j][ch];
          al[j] = (short)dzl[k0 + 4 * kq + j][ch];
        }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
          s4 bv;  // B column: channel of h1
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[j] = (short)a1s[k0 + 4 * kq + j][ni * 16 + row];
          acc2[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bv, acc2[mi][ni], 0, 0, 0);
          acc2[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bv, acc2[mi][ni], 0, 0, 0);
        }
      }
    }
    // dh1 = dz2 W2 (K = 128 channels, hi and lo); wave w takes rows 16w ..
    // 16w+15; dz1 = dh1 where z1 > 0 (h1 > 0), into the h2 buffer (h2 is
    // no longer read)
    {
      f4 acc1[4];
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc1[ni] = f4{0.f, 0.f, 0.f, 0.f};
      const int m = w * 16 + row;
#pragma unroll 2
      for (int k0 = 0; k0 < H2; k0 += 16) {
        s4 ah, al;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          ah[j] = (short)dzh[m][k0 + 4 * kq + j];
          al[j] = (short)dzl[m][k0 + 4 * kq + j];
        }
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
          s4 bv;  // B[i][k] = W2[i][k], column k = channel of h1
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[j] = (short)n.w2h[(size_t)(k0 + 4 * kq + j) * H1 + ni * 16 + row];
          acc1[ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bv, acc1[ni], 0, 0, 0);
          acc1[ni] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bv, acc1[ni], 0, 0, 0);
        }
      }
      __syncthreads();  // every wave is done with h2 before dz1 overwrites it
#pragma unroll
      for (int ni = 0; ni < 4; ++ni)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int mm = w * 16 + 4 * kq + v, k = ni * 16 + row;
          dz1s[mm][k] = from_bf16(a1s[mm][k]) > 0.f ? acc1[ni][v] : 0.f;  // z1 > 0
        }
    }
    __syncthreads();
    // dW1 += dz1^T x, db1 += dz1 (thread < 64: channel tid, rows in order)
    if (tid < H1) {
      for (int mm = 0; mm < nr; ++mm) {
        const float dz = dz1s[mm][tid];
        gW1[0] = __builtin_fmaf(dz, xs[mm][0], gW1[0]);
        gW1[1] = __builtin_fmaf(dz, xs[mm][1], gW1[1]);
        gW1[2] = __builtin_fmaf(dz, xs[mm][2], gW1[2]);
        gb1 += dz;
      }
    }
    __syncthreads();  // buffers are rewritten by the next tile
  }
  // the record: dW2 from the accumulators, D[4 kq + v][row] of each tile
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (2 * w + mi) * 16 + 4 * kq + v, k = ni * 16 + row;
        part[oW2 + i * H1 + k] = acc2[mi][ni][v];
      }
  // db2: the two row halves in a fixed order
  {
    float* red = reinterpret_cast<float*>(u2);
    red[tid] = gb2;
    __syncthreads();
    if (tid < H2) part[ob2 + tid] = red[tid] + red[tid + 128];
  }
  if (tid < H1) {
    part[oW1 + tid * 3 + 0] = gW1[0];
    part[oW1 + tid * 3 + 1] = gW1[1];
    part[oW1 + tid * 3 + 2] = gW1[2];
    part[ob1 + tid] = gb1;
  }
}

// encoder gradient: fixed-order sum of the per-object records
__global__ __launch_bounds__(256) void k_pn_reduce(Net n, float* grad) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kEnc) return;
  float acc = 0.f;
  for (int o = 0; o < n.n_obj; ++o) acc += n.part[(size_t)o * kEnc + e];
  grad[e] = acc / (float)n.n_obj;  // the encoder parameters come first in the flat array
}

__global__ __launch_bounds__(256) void k_pn_adam(float* p, float* m, float* v, const float* g, long long cnt,
                                                  float lr, float b1, float b2, float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= cnt) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace pn

}  // namespace asicp

// ---------------------------------------------------------------------------
// C ABI
namespace {

using namespace asicp;
using namespace asicp::pn;

thread_local std::string pn_err;
asicp_status pn_fail(asicp_status st, const std::string& m) {
  pn_err = m;
  return st;
}

// Runs the body of an entry point so that no C++ exception crosses the C ABI:
// host memory exhaustion in a container or a message string becomes
// ASICP_E_HOST.
template <class F>
asicp_status guarded(F&& body) noexcept {
  try {
    return body();
  } catch (...) {
    pn_err.clear();
    try {
      pn_err = "host-side failure (out of host memory)";
    } catch (...) {
    }
    return ASICP_E_HOST;
  }
}

// The forward pass uses only the buffers up to `out`; fwd_total is their size.
struct PnLayout {
  size_t w2h, w3h, off, com, pool, head, out, dout, dhead, part, lpart, fwd_total, total;
};

PnLayout pn_layout(int n_obj, int n_pre, int n_seed) {
  const Params P = layout(n_pre, n_seed);
  PnLayout L;
  size_t c = 0;
  auto bump = [&c](size_t bytes) { const size_t o = c; c += (bytes + 255) & ~(size_t)255; return o; };
  L.w2h = bump(2 * (size_t)H2 * H1);
  L.w3h = bump(2 * (size_t)H3 * H2);
  L.off = bump(4 * (size_t)(n_obj + 1));
  L.com = bump(16 * (size_t)n_obj);
  L.pool = bump(8 * (size_t)n_obj * H3);
  L.head = bump(4 * (size_t)n_obj * 1024);
  L.out = bump(4 * (size_t)n_obj * P.O);
  L.fwd_total = c;
  L.dout = bump(4 * (size_t)n_obj * P.O);
  L.dhead = bump(4 * (size_t)n_obj * 768);
  L.part = bump(4 * (size_t)n_obj * kEnc);
  L.lpart = bump(4 * (size_t)n_obj * n_pre);
  L.total = c;
  return L;
}

asicp_status pn_check(int n_obj, int n_pre, int n_seed) {
  if (n_obj < 1 || n_obj > 65536) return pn_fail(ASICP_E_INVALID, "n_obj must be in 1..65536");
  if (n_pre < 1 || n_seed < 1 || n_pre * n_seed * 7 > 1024)
    return pn_fail(ASICP_E_INVALID, "n_pre * n_seed * 7 must be in 7..1024");
  return ASICP_OK;
}

// validates the offsets (host) and fills the network descriptor; uploads the
// offsets with the library's kernel-argument uploader
asicp_status pn_setup(Net& n, const float* params, int n_pre, int n_seed, int n_obj, const int32_t* off,
                      const float* x, const float* y, const float* z, void* ws, size_t ws_bytes,
                      hipStream_t hs, int* max_chunks, bool forward_only = false) {
  asicp_status st = pn_check(n_obj, n_pre, n_seed);
  if (st != ASICP_OK) return st;
  if (!params || !off || !x || !y || !z || !ws) return pn_fail(ASICP_E_INVALID, "NULL pointer argument");
  if (off[0] != 0) return pn_fail(ASICP_E_INVALID, "offsets must start at 0");
  int mc = 0;
  for (int o = 0; o < n_obj; ++o) {
    const long long m = (long long)off[o + 1] - off[o];
    if (m < 1 || m > (1 << 22)) return pn_fail(ASICP_E_INVALID, "object " + std::to_string(o) + " must have 1..4194304 points");
    mc = std::max(mc, (int)((m + kPts - 1) / kPts));
  }
  const PnLayout L = pn_layout(n_obj, n_pre, n_seed);
  if (ws_bytes < (forward_only ? L.fwd_total : L.total)) return pn_fail(ASICP_E_INVALID, "workspace too small");
  char* b = static_cast<char*>(ws);
  n.prm = params;
  n.w2h = reinterpret_cast<unsigned short*>(b + L.w2h);
  n.w3h = reinterpret_cast<unsigned short*>(b + L.w3h);
  n.off = reinterpret_cast<const int32_t*>(b + L.off);
  n.x = x; n.y = y; n.z = z;
  n.com = reinterpret_cast<float*>(b + L.com);
  n.pool = reinterpret_cast<unsigned long long*>(b + L.pool);
  n.head = reinterpret_cast<float*>(b + L.head);
  n.out = reinterpret_cast<float*>(b + L.out);
  n.dout = forward_only ? nullptr : reinterpret_cast<float*>(b + L.dout);
  n.dhead = forward_only ? nullptr : reinterpret_cast<float*>(b + L.dhead);
  n.part = forward_only ? nullptr : reinterpret_cast<float*>(b + L.part);
  n.n_obj = n_obj; n.n_pre = n_pre; n.n_seed = n_seed; n.n_tgt = 0;
  n.P = layout(n_pre, n_seed);
  (void)hipGetLastError();
  upload_words(b + L.off, off, 4 * (size_t)(n_obj + 1), hs);
  *max_chunks = mc;
  return ASICP_OK;
}

void pn_forward(const Net& n, int mc, float* seeds, float retract, hipStream_t hs) {
  hipLaunchKernelGGL(k_pn_prep, dim3(n.n_obj + 1), dim3(256), 0, hs, n);
  hipLaunchKernelGGL(k_pn_point_fwd, dim3(n.n_obj * mc), dim3(256), 0, hs, n, mc);
  hipLaunchKernelGGL(k_pn_head_fwd, dim3(n.n_obj), dim3(256), 0, hs, n, seeds, n.n_obj * n.n_pre * n.n_seed,
                     retract);
}

asicp_status pn_launched(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return pn_fail(ASICP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return ASICP_OK;
}

// Forward pass and the optional copy of the raw outputs, on a workspace the
// caller or the library provides.
asicp_status pn_forward_call(const float* params, int n_pre, int n_seed, int n_obj, const int32_t* off,
                             const float* x, const float* y, const float* z, float retract, float* seeds,
                             float* raw, void* ws, size_t ws_bytes, bool forward_only, hipStream_t hs) {
  if (!std::isfinite(retract)) return pn_fail(ASICP_E_INVALID, "retract must be finite");
  Net n;
  int mc = 0;
  asicp_status st = pn_setup(n, params, n_pre, n_seed, n_obj, off, x, y, z, ws, ws_bytes, hs, &mc, forward_only);
  if (st != ASICP_OK) return st;
  pn_forward(n, mc, seeds, retract, hs);
  if ((st = pn_launched("proposal forward")) != ASICP_OK) return st;
  if (raw && hipMemcpyAsync(raw, n.out, 4 * (size_t)n_obj * n.P.O, hipMemcpyDeviceToDevice, hs) != hipSuccess)
    return pn_fail(ASICP_E_HIP, "copying the raw outputs failed");
  return ASICP_OK;
}

// Device-resident workspace of asicp_pn_forward_noalloc: every intermediate
// of a forward pass of up to kNoAllocObjects objects.  Each device the
// library runs on holds its own copy until the process ends.  Host code never
// uses the symbol itself (on the host it names a stand-in, not device
// memory): it uses the device address that hipGetSymbolAddress returns,
// looked up once per device and kept in scratch_addr.
constexpr int kNoAllocObjects = 64;
constexpr size_t kNoAllocBytes = 1u << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_addr[kMaxDevices] = {};

asicp_status scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return pn_fail(ASICP_E_HIP, "hipGetDevice failed");
  if (dev >= kMaxDevices) return pn_fail(ASICP_E_INVALID, "device index beyond the library's table (64)");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return pn_fail(ASICP_E_HIP, std::string("hipGetSymbolAddress of the scratch array: ") + hipGetErrorString(e));
    scratch_addr[dev] = p;
  }
  *out = scratch_addr[dev];
  return ASICP_OK;
}

}  // namespace

extern "C" {

const char* asicp_pn_last_error(void) { return pn_err.c_str(); }

int64_t asicp_pn_param_count(int32_t n_pre, int32_t n_seed) {
  if (n_pre < 1 || n_seed < 1 || n_pre * n_seed * 7 > 1024) return -1;
  return layout(n_pre, n_seed).total;
}

asicp_status asicp_pn_workspace_bytes(int32_t n_obj, int32_t n_pre, int32_t n_seed, size_t* bytes) {
  return guarded([&]() -> asicp_status {
    pn_err.clear();
    if (!bytes) return pn_fail(ASICP_E_INVALID, "bytes must not be NULL");
    const asicp_status st = pn_check(n_obj, n_pre, n_seed);
    if (st != ASICP_OK) return st;
    *bytes = pn_layout(n_obj, n_pre, n_seed).total;
    return ASICP_OK;
  });
}

asicp_status asicp_pn_forward(const float* params, int32_t n_pre, int32_t n_seed, int32_t n_obj,
                              const int32_t* off, const float* x, const float* y, const float* z,
                              float retract, float* seeds, float* raw, void* workspace, size_t ws_bytes,
                              void* stream) {
  return guarded([&]() -> asicp_status {
    pn_err.clear();
    return pn_forward_call(params, n_pre, n_seed, n_obj, off, x, y, z, retract, seeds, raw, workspace, ws_bytes,
                           false, static_cast<hipStream_t>(stream));
  });
}

asicp_status asicp_pn_forward_noalloc(const float* params, int32_t n_pre, int32_t n_seed, int32_t n_obj,
                                      const int32_t* off, const float* x, const float* y, const float* z,
                                      float retract, float* seeds, float* raw, void* stream) {
  return guarded([&]() -> asicp_status {
    pn_err.clear();
    asicp_status st = pn_check(n_obj, n_pre, n_seed);
    if (st != ASICP_OK) return st;
    if (n_obj > kNoAllocObjects)
      return pn_fail(ASICP_E_INVALID, "asicp_pn_forward_noalloc takes at most 64 objects per call");
    const size_t need = pn_layout(n_obj, n_pre, n_seed).fwd_total;
    if (need > kNoAllocBytes)
      return pn_fail(ASICP_E_INVALID, "forward pass needs more than the 1 MiB device scratch");
    void* ws = nullptr;
    if ((st = scratch_for_current_device(&ws)) != ASICP_OK) return st;
    return pn_forward_call(params, n_pre, n_seed, n_obj, off, x, y, z, retract, seeds, raw, ws, kNoAllocBytes,
                           true, static_cast<hipStream_t>(stream));
  });
}

asicp_status asicp_pn_loss_grad(const float* params, int32_t n_pre, int32_t n_seed, int32_t n_obj,
                                const int32_t* off, const float* x, const float* y, const float* z,
                                const float* targets, int32_t n_targets, float* loss, float* grad,
                                void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&]() -> asicp_status {
    pn_err.clear();
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (!targets || !loss || !grad) return pn_fail(ASICP_E_INVALID, "NULL pointer argument");
    if (n_targets < 1 || n_targets > 4096) return pn_fail(ASICP_E_INVALID, "n_targets must be in 1..4096");
    Net n;
    int mc = 0;
    asicp_status st = pn_setup(n, params, n_pre, n_seed, n_obj, off, x, y, z, workspace, ws_bytes, hs, &mc);
    if (st != ASICP_OK) return st;
    n.n_tgt = n_targets;
    pn_forward(n, mc, nullptr, 0.f, hs);
    float* lpart = reinterpret_cast<float*>(static_cast<char*>(workspace) + pn_layout(n_obj, n_pre, n_seed).lpart);
    const int pairs = n_obj * n_pre;
    hipLaunchKernelGGL(k_pn_loss, dim3(pairs), dim3(64), 0, hs, n, targets, lpart);
    hipLaunchKernelGGL(k_pn_loss_sum, dim3((n_obj + 63) / 64), dim3(64), 0, hs, n, lpart, loss);
    hipLaunchKernelGGL(k_pn_head_bwd, dim3(n_obj), dim3(256), 0, hs, n);
    const long long head_elems = (long long)HH * H3 + HH + (long long)HH * HH + HH + (long long)n.P.O * HH + n.P.O;
    hipLaunchKernelGGL(k_pn_head_wgrad, dim3((unsigned)((head_elems + 255) / 256)), dim3(256), 0, hs, n, grad);
    hipLaunchKernelGGL(k_pn_point_bwd, dim3(n_obj), dim3(256), 0, hs, n);
    hipLaunchKernelGGL(k_pn_reduce, dim3((kEnc + 255) / 256), dim3(256), 0, hs, n, grad);
    return pn_launched("proposal loss and gradient");
  });
}

asicp_status asicp_pn_adam(float* params, float* m, float* v, const float* grad, int64_t count, float lr,
                           float beta1, float beta2, float eps, int32_t step, void* stream) {
  return guarded([&]() -> asicp_status {
    pn_err.clear();
    if (!params || !m || !v || !grad) return pn_fail(ASICP_E_INVALID, "NULL pointer argument");
    if (count < 1 || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
      return pn_fail(ASICP_E_INVALID, "bad Adam settings");
    const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(k_pn_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       params, m, v, grad, (long long)count, lr, beta1, beta2, eps, c1, c2);
    return pn_launched("Adam step");
  });
}

}  // extern "C"
