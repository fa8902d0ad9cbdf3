// k_minibatch.hip -- mini-batch of the object cloud per iteration (Algorithm 1
// "select a mini-batch from R"; size schedule of Table I): one batch per
// object and iteration, shared by the object's particles.  The batch is
// {perm(j) : j < m_k} for a keyed permutation of the cloud's indices: a
// 4-round balanced Feistel network whose round function is SplitMix64
// (Steele, Lea and Flood, 2014), cycle-walked into [0, M).  Points outside
// the batch get |r|^2 = 1e30 in a copy of the MFMA-ready cloud, so the
// nearest-neighbour kernels never pick them; the chunk boxes of the whole
// cloud remain valid lower bounds.
#include "nn_core.h"

namespace asicp {

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ long long batch_perm(long long j, long long M, unsigned long long key) {
  int bits = 2;
  while ((1ll << bits) < M) ++bits;
  if (bits & 1) ++bits;
  const int hb = bits / 2;
  const unsigned long long mask = (1ull << hb) - 1ull;
  unsigned long long x = (unsigned long long)j;
  do {
    unsigned long long L = x >> hb, R = x & mask;
    for (unsigned long long r = 0; r < 4; ++r) {
      const unsigned long long F = splitmix64(key ^ (r << 56) ^ R) & mask;
      const unsigned long long nL = R, nR = L ^ F;
      L = nL;
      R = nR;
    }
    x = (L << hb) | R;
  } while (x >= (unsigned long long)M);
  return (long long)x;
}

// grid: (ceil(max M / 256), n_obj)
__global__ __launch_bounds__(256) void k_batch_mark(Dev d, int k, double frac) {
  const int o = blockIdx.y;
  const ObjInfo& oi = d.objs[o];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= oi.m) return;
  long long mb = (long long)ceil((double)oi.m * frac);
  mb = mb < 1 ? 1 : (mb > oi.m ? oi.m : mb);
  const unsigned long long key =
      splitmix64(splitmix64(d.seed) ^ ((unsigned long long)(unsigned)k << 20) ^ (unsigned long long)(unsigned)o);
  const long long p = (mb == oi.m) ? j : batch_perm(j, oi.m, key);
  d.batch_mark[oi.r_begin + p] = (j < mb) ? 1 : 0;
}

// grid: (ceil(max padded M / 256), n_obj)
__global__ __launch_bounds__(256) void k_batch_prep(Dev d) {
  const int o = blockIdx.y;
  const ObjInfo& oi = d.objs[o];
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= oi.ntg * 64) return;
  const size_t g = (size_t)oi.prep_tg_begin * 64 + k;
  const int orig = d.obj_perm[g];
  const float4 p = d.obj_pts[g];
  float* pf = reinterpret_cast<float*>(d.obj_prep_mb + (size_t)oi.prep_tg_begin * 64);
  if (orig >= 0 && d.batch_mark[oi.r_begin + orig]) {
    prep_store(pf, k, -2.f * p.x, -2.f * p.y, -2.f * p.z,
               __builtin_fmaf(p.z, p.z, __builtin_fmaf(p.y, p.y, p.x * p.x)));
  } else {
    prep_store(pf, k, 0.f, 0.f, 0.f, kDummyNorm);
  }
}

void launch_minibatch(const Dev& d, int k, double frac, hipStream_t s) {
  hipLaunchKernelGGL(k_batch_mark, dim3((d.max_m + 255) / 256, d.n_obj), dim3(256), 0, s, d, k, frac);
  hipLaunchKernelGGL(k_batch_prep, dim3((d.max_m_pad + 255) / 256, d.n_obj), dim3(256), 0, s, d);
}

}  // namespace asicp
